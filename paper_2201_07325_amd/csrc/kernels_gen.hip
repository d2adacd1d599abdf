// Kernel-entry generation: pair-tile assembly, the ID matrix with its proxy rows, the
// stand-alone block generator and the exact on-the-fly matvec.
//
// Entries follow Section 3 (eqs. disc1, disc3, comb_ref) with plain smooth weights:
//   A~_ii = 1/2,  A~_ij = sqrt(w_i) K(x_i, x_j) sqrt(w_j),
//   K(x, y) = e^{ik r} / (4 pi r^3) * [ (1 - ik r) (x - y).n(y) - i eta r^2 ],  r = |x - y|.
// All generators are VALU-bound (one sine-cosine pair and one reciprocal square root per
// entry); work is split into 64x64 units so that a workgroup of 256 threads writes whole
// columns (consecutive threads -> consecutive rows, coalesced stores).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <vector>
#include <string>

#include "kernels.hpp"

namespace fmmlu {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

// 1/sqrt(x) for x > 0 (every squared distance between distinct points): the hardware
// estimate y0, then one second-order correction from the binomial series
// 1/sqrt(1 - e) = 1 + e/2 + 3e^2/8 + ... with e = 1 - x y0^2, whose truncation (about
// 5e^3/16) is far below a rounding error for the estimate's relative error.
__device__ inline double rsqrt_pos(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y0, y0, 1.0);
  return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// Sine and cosine of the kernel phase x = k r. Below kPhaseFast: Cody-Waite reduction by
// pi/2 with fused multiply-adds (x - q hi exact to one rounding, then the tail lo of pi/2) to
// |y| <= pi/4, the Taylor series of sin to y^15 and of cos to y^16 (truncation below 7e-17
// relative on that interval), and the quadrant q mod 4. Both series are sums over the powers
// of z = y^2, formed once and shared: each term is one multiply-add of a coefficient and a
// ready power, smallest term first, so no coefficient has to be copied into an accumulator
// register first (as the addend of a Horner step would be). At or beyond kPhaseFast
// sincos_phase calls the library's routine.
constexpr double kPhaseFast = 1048576.0;

// sin y and cos y of the reduced argument y = x - q pi/2, and q mod 4 (returned), so that
// e^{ix} = i^q (cos y + i sin y); |x| < kPhaseFast.
__device__ inline int sincos_phase_quadrant(double x, double* sy_out, double* cy_out) {
  constexpr double kTwoOverPi = 0.63661977236758134308;
  constexpr double kPio2Hi = 1.5707963267948965580;   // nearest double to pi/2
  constexpr double kPio2Lo = 6.123233995736766036e-17;  // pi/2 - kPio2Hi
  const double q = rint(x * kTwoOverPi);
  double y = fma(-q, kPio2Hi, x);
  y = fma(-q, kPio2Lo, y);
  const double z = y * y;
  const double z2 = z * z, z3 = z2 * z, z4 = z2 * z2, z5 = z4 * z, z6 = z4 * z2, z7 = z4 * z3;
  // sin y = y + y z (-1/3! + z/5! - ... - z^6/15!)
  double ps = -7.6471637318198164759e-13 * z6;       // -1/15!
  ps = fma(1.6059043836821614599e-10, z5, ps);       //  1/13!
  ps = fma(-2.5052108385441718775e-08, z4, ps);      // -1/11!
  ps = fma(2.7557319223985890653e-06, z3, ps);       //  1/9!
  ps = fma(-1.9841269841269841270e-04, z2, ps);      // -1/7!
  ps = fma(8.3333333333333333333e-03, z, ps);        //  1/5!
  ps = ps - 1.6666666666666666667e-01;               // -1/3!
  const double sy = fma(ps * z, y, y);
  // cos y = 1 + z (-1/2! + z/4! - ... + z^7/16!)
  double pc = 4.7794773323873852974e-14 * z7;        //  1/16!
  pc = fma(-1.1470745597729724714e-11, z6, pc);      // -1/14!
  pc = fma(2.0876756987868098979e-09, z5, pc);       //  1/12!
  pc = fma(-2.7557319223985890653e-07, z4, pc);      // -1/10!
  pc = fma(2.4801587301587301587e-05, z3, pc);       //  1/8!
  pc = fma(-1.3888888888888888889e-03, z2, pc);      // -1/6!
  pc = fma(4.1666666666666666667e-02, z, pc);        //  1/4!
  pc = pc - 0.5;                                     // -1/2!
  const double cy = fma(pc, z, 1.0);
  *sy_out = sy;
  *cy_out = cy;
  return (int)q & 3;  // |q| < 2^20: exact in an int
}

// sin x and cos x for |x| < kPhaseFast
__device__ inline void sincos_phase_reduced(double x, double* sn, double* cs) {
  double sy, cy;
  const int quad = sincos_phase_quadrant(x, &sy, &cy);
  const double s0 = (quad & 1) ? cy : sy, c0 = (quad & 1) ? sy : cy;
  *sn = (quad & 2) ? -s0 : s0;
  *cs = ((quad + 1) & 2) ? -c0 : c0;
}

// (u + i v) i^q for q in 0..3
__device__ inline void rotate_quadrant(int q, double& u, double& v) {
  const double u0 = u;
  u = (q & 1) ? -v : u;
  v = (q & 1) ? u0 : v;
  if (q & 2) {
    u = -u;
    v = -v;
  }
}

__device__ inline void sincos_phase(double x, double* sn, double* cs) {
  if (!(fabs(x) < kPhaseFast)) {
    sincos(x, sn, cs);
    return;
  }
  sincos_phase_reduced(x, sn, cs);
}

// A~[i, j] for tree positions i, j
__device__ inline zd cfie_entry(const double* __restrict__ p, int64_t n, double k, double eta,
                                int64_t i, int64_t j) {
  if (i == j) return zd{0.5, 0.0};
  double dx = p[i] - p[j], dy = p[n + i] - p[n + j], dz = p[2 * n + i] - p[2 * n + j];
  double r2 = dx * dx + dy * dy + dz * dz;
  double ir = rsqrt_pos(r2);
  double r = r2 * ir;
  double dn = dx * p[3 * n + j] + dy * p[4 * n + j] + dz * p[5 * n + j];
  double s, c;
  sincos_phase(k * r, &s, &c);
  double a = dn, b = k * r * dn + eta * r2;
  double f = p[6 * n + i] * p[6 * n + j] * kInv4Pi * (ir * ir * ir);
  return zd{(c * a + s * b) * f, (s * a - c * b) * f};
}

// d/dk of A~[i, j] at fixed eta
__device__ inline zd cfie_entry_dk(const double* __restrict__ p, int64_t n, double k, double eta,
                                   int64_t i, int64_t j) {
  if (i == j) return zd{0.0, 0.0};
  double dx = p[i] - p[j], dy = p[n + i] - p[n + j], dz = p[2 * n + i] - p[2 * n + j];
  double r2 = dx * dx + dy * dy + dz * dz;
  double ir = rsqrt_pos(r2);
  double r = r2 * ir;
  double dn = dx * p[3 * n + j] + dy * p[4 * n + j] + dz * p[5 * n + j];
  double s, c;
  sincos_phase(k * r, &s, &c);
  // k e^{ikr} dn / (4 pi r)  +  eta r e^{ikr} / (4 pi r) = e^{ikr} (k dn + eta r) / (4 pi r)
  double f = p[6 * n + i] * p[6 * n + j] * kInv4Pi * ir;
  double a = k * dn + eta * r;
  return zd{c * a * f, s * a * f};
}

// d/deta of A~[i, j] = -i sqrt(w_i w_j) G
__device__ inline zd cfie_entry_deta(const double* __restrict__ p, int64_t n, double k,
                                     int64_t i, int64_t j) {
  if (i == j) return zd{0.0, 0.0};
  double dx = p[i] - p[j], dy = p[n + i] - p[n + j], dz = p[2 * n + i] - p[2 * n + j];
  double r2 = dx * dx + dy * dy + dz * dz;
  double ir = rsqrt_pos(r2);
  double s, c;
  sincos_phase(k * (r2 * ir), &s, &c);
  double f = p[6 * n + i] * p[6 * n + j] * kInv4Pi * ir;
  return zd{s * f, -c * f};
}

// correction factor 1 + a_ij of a listed pair (1 when the pair is not listed or i == j)
__device__ inline double corr_factor(const DevCorr& c, int64_t i, int64_t j) {
  if (!c.rptr || i == j) return 1.0;
  int64_t lo = c.rptr[i], hi = c.rptr[i + 1];
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (c.rcol[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && c.rcol[lo] == j) ? 1.0 + c.ra[lo] : 1.0;
}

// A~[i, j] with the quadrature corrections of the system
__device__ inline zd entry(const DevGeom& g, int64_t i, int64_t j) {
  return zscale(cfie_entry(g.p, g.n, g.k, g.eta, i, j), corr_factor(g.corr, i, j));
}

template <class Task>
__device__ inline int find_task(const Task* __restrict__ t, int n, int64_t u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (t[mid].unit_begin <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------------------
template <class ST, class DT>
__global__ void __launch_bounds__(256) assemble_kernel(DevGeom g, const AsmTask* __restrict__ tasks,
                                                       int ntasks, const int32_t* __restrict__ slot,
                                                       const int32_t* __restrict__ idx,
                                                       const int64_t* __restrict__ dof,
                                                       const AsmSrc* __restrict__ table,
                                                       const ST* __restrict__ src, DT* __restrict__ dst,
                                                       const int32_t* __restrict__ utask) {
  const int64_t u = blockIdx.x;
  const int ti = utask ? utask[u] : find_task(tasks, ntasks, u);
  const AsmTask t = tasks[ti];
  const int64_t lu = u - t.unit_begin;
  const int nbr = (t.nr + 63) >> 6;
  const int bi = (int)(lu % nbr), bj = (int)(lu / nbr);
  const int i = bi * 64 + (threadIdx.x & 63);
  if (i >= t.nr) return;
  const int rs = slot[t.rmap_off + i];
  const int ri = idx[t.rmap_off + i];
  const int64_t rd = dof[t.rdof_off + i];
  // the thread's 16 columns j0 + 4 jj in two rounds of eight: column maps, then source table
  // entries, then the values, each issued for the round's eight columns before the next
  // (three dependent reads per entry: eight of each in flight instead of one)
  const int j0 = bj * 64 + (threadIdx.x >> 6);
  const int nj = min(16, (t.nc - j0 + 3) >> 2);
  for (int h = 0; h < 2; ++h) {
    constexpr int R = 8;
    const int jb = R * h;
    if (jb >= nj) break;
    int cs[R], ci[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool ok = jb + q < nj;
      cs[q] = ok ? slot[t.cmap_off + j0 + 4 * (jb + q)] : 0;
      ci[q] = ok ? idx[t.cmap_off + j0 + 4 * (jb + q)] : 0;
    }
    int64_t so[R];
    int32_t sl[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const AsmSrc sr = jb + q < nj ? table[t.tab_off + (int64_t)rs * t.nsc + cs[q]] : AsmSrc{-1, 0, 0};
      so[q] = sr.off;
      sl[q] = sr.ld;
    }
    ST sv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) sv[q] = (jb + q < nj && so[q] >= 0) ? src[so[q] + ri + (int64_t)ci[q] * sl[q]] : ST{};
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (jb + q >= nj) break;
      const int j = j0 + 4 * (jb + q);
      const zd v = so[q] >= 0 ? widen(sv[q]) : entry(g, rd, dof[t.cdof_off + j]);
      dst[t.out_off + i + (int64_t)j * t.ld] = narrow<DT>(v);
    }
  }
}

// ---------------------------------------------------------------------------------------
template <class PT>
__global__ void __launch_bounds__(256) idmatrix_kernel(DevGeom g, const IdTask* __restrict__ tasks,
                                                       int ntasks, const QSeg* __restrict__ segs,
                                                       const int64_t* __restrict__ dof,
                                                       const PT* __restrict__ pool) {
  const int64_t u = blockIdx.x;
  const int ti = find_task(tasks, ntasks, u);
  const IdTask t = tasks[ti];
  const int64_t lu = u - t.unit_begin;
  const int nbr = (t.rows + 63) >> 6;
  const int bi = (int)(lu % nbr), bj = (int)(lu / nbr);
  const int i = bi * 64 + (threadIdx.x & 63);
  if (i >= t.rows) return;
  const double* p = g.p;
  const int64_t n = g.n;
  zd* out = t.M;
  if (i < 2 * t.nq) {
    const bool transposed = i >= t.nq;
    const int iq = transposed ? i - t.nq : i;
    // segment containing row iq
    int lo = 0, hi = t.nseg - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (segs[t.seg_off + mid].row0 <= iq)
        lo = mid;
      else
        hi = mid - 1;
    }
    const QSeg sg = segs[t.seg_off + lo];
    const int li = sg.live[iq - sg.row0];
    if (sg.tile_qb < 0) {
      // spill-over owner without a stored tile: corrected kernel values
      const int64_t q = sg.gdof[li];
      for (int jj = 0; jj < 16; ++jj) {
        const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
        if (j >= t.m) break;
        const int64_t b = dof[t.dof_off + j];
        out[i + (int64_t)j * t.rows] = transposed ? entry(g, b, q) : entry(g, q, b);
      }
      return;
    }
    // all 16 reads in flight before the writes
    PT vals[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
      vals[jj] = PT{};
      if (j < t.m)
        vals[jj] = transposed ? pool[sg.tile_bq + j + (int64_t)li * t.m] : pool[sg.tile_qb + li + (int64_t)j * sg.ld];
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
      if (j < t.m) out[i + (int64_t)j * t.rows] = widen(vals[jj]);
    }
    return;
  }
  // proxy row: Fibonacci point l on the sphere of the given centre and radius
  const bool incoming = i >= 2 * t.nq + t.ngamma;
  const int l = incoming ? i - 2 * t.nq - t.ngamma : i - 2 * t.nq;
  const double golden = M_PI * (3.0 - sqrt(5.0));
  const double z = 1.0 - (2.0 * l + 1.0) / t.ngamma;
  const double phi = l * golden;
  const double rr = sqrt(fmax(0.0, 1.0 - z * z));
  double sp, cp;
  sincos(phi, &sp, &cp);
  const double yx = t.cx + t.radius * (rr * cp);
  const double yy = t.cy + t.radius * (rr * sp);
  const double yz = t.cz + t.radius * z;
  for (int jj = 0; jj < 16; ++jj) {
    const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
    if (j >= t.m) break;
    const int64_t q = dof[t.dof_off + j];
    const double dx = yx - p[q], dy = yy - p[n + q], dz = yz - p[2 * n + q];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt_pos(r2);
    const double r = r2 * ir;
    double s, c;
    sincos_phase(g.k * r, &s, &c);
    const double sw = p[6 * n + q] * t.wgamma;
    zd v;
    if (incoming) {
      // G(x_j, y_l) sqrt(w_j)
      const double f = sw * kInv4Pi * ir;
      v = zd{c * f, s * f};
    } else {
      // K(y_l, x_j) sqrt(w_j), source normal n_j
      const double dn = dx * p[3 * n + q] + dy * p[4 * n + q] + dz * p[5 * n + q];
      const double a = dn, b = g.k * r * dn + g.eta * r2;
      const double f = sw * kInv4Pi * (ir * ir * ir);
      v = zd{(c * a + s * b) * f, (s * a - c * b) * f};
    }
    out[i + (int64_t)j * t.rows] = v;
  }
}

// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) block_kernel(DevGeom g, const int64_t* __restrict__ rows,
                                                    int64_t nr, const int64_t* __restrict__ cols,
                                                    int64_t nc, zd* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nr * nc) return;
  const int64_t i = e % nr, j = e / nr;
  out[e] = entry(g, rows[i], cols[j]);
}

// ---------------------------------------------------------------------------------------
// One source j of the exact matvec for the thread's target i, added to (are, aim) without the
// target's weight sqrt(w_i), which the caller applies once to the sum. sp holds the sources'
// coordinates and normals, sx the sources' x_j sqrt(w_j) / (4 pi); the entry over those
// weights is (A + iB) f. FAST (every phase below kPhaseFast): A + iB is formed from the
// reduced sine and cosine and turned by the phase's quadrant once, instead of selecting and
// negating sine and cosine.
template <int OP, bool FAST>
__device__ inline void matvec_pair(const DevGeom& g, const double (&xi)[6], const double (*sp)[256],
                                   const zd* sx, int jj, double& are, double& aim) {
  const double dx = xi[0] - sp[0][jj], dy = xi[1] - sp[1][jj], dz = xi[2] - sp[2][jj];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt_pos(r2);
  const double r = r2 * ir;
  const double kr = g.k * r;
  double s, c;
  int quad = 0;
  if (FAST)
    quad = sincos_phase_quadrant(kr, &s, &c);
  else
    sincos_phase(kr, &s, &c);
  double A, B, f;
  if (OP == 0) {
    // e^{ikr} (dn - i b)
    const double dn = dx * sp[3][jj] + dy * sp[4][jj] + dz * sp[5][jj];
    const double b = kr * dn + g.eta * r2;
    f = ir * ir * ir;
    A = c * dn + s * b;
    B = s * dn - c * b;
  } else if (OP == 1) {
    // conj(A~[j, i]) = e^{-ikr} (dn + i b): target j, source i with normal n_i;
    // d = x_j - x_i = -(dx, dy, dz)
    const double dn = -(dx * xi[3] + dy * xi[4] + dz * xi[5]);
    const double b = kr * dn + g.eta * r2;
    f = ir * ir * ir;
    A = c * dn + s * b;
    B = c * b - s * dn;
    quad = (4 - quad) & 3;
  } else if (OP == 2) {
    // e^{ikr} a
    const double dn = dx * sp[3][jj] + dy * sp[4][jj] + dz * sp[5][jj];
    const double a = g.k * dn + g.eta * r;
    f = ir;
    A = c * a;
    B = s * a;
  } else {
    // -i e^{ikr}
    f = ir;
    A = s;
    B = -c;
  }
  if (FAST) rotate_quadrant(quad, A, B);
  const zd xv = sx[jj];
  const double xr = xv.re * f, xm = xv.im * f;
  are = fma(A, xr, are);
  are = fma(-B, xm, are);
  aim = fma(A, xm, aim);
  aim = fma(B, xr, aim);
}

// Exact matvec: each workgroup owns 256 target rows and streams one slice of the sources
// through LDS; slices (grid.y) write partial sums that a second pass adds in a fixed order.
// op 0: y = A~ x; 1: y = A~^H x; 2: y = dA~/dk x; 3: y = dA~/deta x. Vectors in tree order.
// Source tiles start at multiples of 256 (the slice length is one), so the diagonal entry of
// every target of the workgroup lies in the one tile that starts at the workgroup's first
// target, at position threadIdx.x; only that tile's loop tests for it. FAST: every phase
// k r of the launch is known to lie below kPhaseFast (no per-entry range test).
template <int OP, bool FAST>
__global__ void __launch_bounds__(256) matvec_kernel(DevGeom g, const zd* __restrict__ x, zd* __restrict__ part,
                                                     int64_t slice) {
  __shared__ double sp[6][256];
  __shared__ zd sx[256];
  const int64_t n = g.n;
  const double* p = g.p;
  const int64_t ib = (int64_t)blockIdx.x * 256, i = ib + threadIdx.x;
  const bool live = i < n;
  double xi[6];
  for (int a = 0; a < 6; ++a) xi[a] = live ? p[a * n + i] : 0.0;
  const double wi = live ? p[6 * n + i] : 0.0;
  double are = 0.0, aim = 0.0, dre = 0.0, dim = 0.0;
  const int64_t jbeg = (int64_t)blockIdx.y * slice, jend = min(n, jbeg + slice);
  for (int64_t j0 = jbeg; j0 < jend; j0 += 256) {
    __syncthreads();
    const int64_t jl = j0 + threadIdx.x;
    for (int a = 0; a < 6; ++a) sp[a][threadIdx.x] = jl < jend ? p[a * n + jl] : 0.0;
    if (jl < jend) {
      const zd xj = x[jl];
      const double wj = p[6 * n + jl] * kInv4Pi;
      sx[threadIdx.x] = zd{xj.re * wj, xj.im * wj};
    } else {
      sx[threadIdx.x] = zd{0.0, 0.0};
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(256, jend - j0);
    if (!live) continue;
    if (j0 == ib) {
      for (int jj = 0; jj < cnt; ++jj) {
        if (jj == (int)threadIdx.x) {
          if (OP <= 1) {
            const zd xd = x[i];  // sx holds the weighted values
            dre = 0.5 * xd.re;
            dim = 0.5 * xd.im;
          }
          continue;
        }
        matvec_pair<OP, FAST>(g, xi, sp, sx, jj, are, aim);
      }
    } else {
#pragma unroll 2
      for (int jj = 0; jj < cnt; ++jj) matvec_pair<OP, FAST>(g, xi, sp, sx, jj, are, aim);
    }
  }
  if (live) part[(int64_t)blockIdx.y * n + i] = zd{fma(wi, are, dre), fma(wi, aim, dim)};
}

// The corrections' share of the exact product: the listed entries beyond their kernel value,
// a_ij K_ij (or its derivative), added to y in the order of the lists. op 1 walks the lists
// by column for the conjugate transpose.
template <int OP>
__global__ void __launch_bounds__(256) matvec_corr_kernel(DevGeom g, const zd* __restrict__ x, zd* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= g.n) return;
  const DevCorr& c = g.corr;
  zd acc = y[i];
  if (OP == 1) {
    for (int64_t e = c.cptr[i]; e < c.cptr[i + 1]; ++e) {
      const int64_t r = c.crow[e];
      zfmac(acc, zscale(cfie_entry(g.p, g.n, g.k, g.eta, r, i), c.ca[e]), x[r]);
    }
  } else {
    for (int64_t e = c.rptr[i]; e < c.rptr[i + 1]; ++e) {
      const int64_t j = c.rcol[e];
      const zd v = OP == 0 ? cfie_entry(g.p, g.n, g.k, g.eta, i, j)
                 : OP == 2 ? cfie_entry_dk(g.p, g.n, g.k, g.eta, i, j)
                           : cfie_entry_deta(g.p, g.n, g.k, i, j);
      zfma(acc, zscale(v, c.ra[e]), x[j]);
    }
  }
  y[i] = acc;
}

__global__ void __launch_bounds__(256) matvec_sum_kernel(const zd* __restrict__ part, int64_t n, int nslice,
                                                         zd* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  zd s = part[i];
  for (int q = 1; q < nslice; ++q) s = zadd(s, part[(int64_t)q * n + i]);
  y[i] = s;
}

}  // namespace

void launch_assemble(const DevGeom& g, const AsmTask* tasks, int ntasks, int64_t nunits,
                     const int32_t* slot, const int32_t* idx, const int64_t* dof,
                     const AsmSrc* table, const void* src_pool, bool src32, void* dst_pool, bool dst32,
                     hipStream_t st, const int32_t* utask) {
  if (ntasks <= 0 || nunits <= 0) return;
  const dim3 gr((unsigned)nunits), b(256);
  if (!src32 && !dst32)
    hipLaunchKernelGGL((assemble_kernel<zd, zd>), gr, b, 0, st, g, tasks, ntasks, slot, idx, dof, table,
                       static_cast<const zd*>(src_pool), static_cast<zd*>(dst_pool), utask);
  else if (src32 && dst32)
    hipLaunchKernelGGL((assemble_kernel<zf, zf>), gr, b, 0, st, g, tasks, ntasks, slot, idx, dof, table,
                       static_cast<const zf*>(src_pool), static_cast<zf*>(dst_pool), utask);
  else if (src32)
    hipLaunchKernelGGL((assemble_kernel<zf, zd>), gr, b, 0, st, g, tasks, ntasks, slot, idx, dof, table,
                       static_cast<const zf*>(src_pool), static_cast<zd*>(dst_pool), utask);
  else
    hipLaunchKernelGGL((assemble_kernel<zd, zf>), gr, b, 0, st, g, tasks, ntasks, slot, idx, dof, table,
                       static_cast<const zd*>(src_pool), static_cast<zf*>(dst_pool), utask);
  FMMLU_HIP(hipGetLastError());
}

void launch_build_idmatrix(const DevGeom& g, const IdTask* tasks, int ntasks, int64_t nunits,
                           const QSeg* segs, const int64_t* dof, const void* pool, bool pool32, hipStream_t st) {
  if (ntasks <= 0 || nunits <= 0) return;
  if (pool32)
    hipLaunchKernelGGL(idmatrix_kernel<zf>, dim3((unsigned)nunits), dim3(256), 0, st, g, tasks, ntasks, segs, dof,
                       static_cast<const zf*>(pool));
  else
    hipLaunchKernelGGL(idmatrix_kernel<zd>, dim3((unsigned)nunits), dim3(256), 0, st, g, tasks, ntasks, segs, dof,
                       static_cast<const zd*>(pool));
  FMMLU_HIP(hipGetLastError());
}

void launch_block(const DevGeom& g, const int64_t* rows, int64_t nr, const int64_t* cols,
                  int64_t nc, zd* out, hipStream_t st) {
  int64_t tot = nr * nc;
  if (tot <= 0) return;
  hipLaunchKernelGGL(block_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, rows,
                     nr, cols, nc, out);
  FMMLU_HIP(hipGetLastError());
}

namespace {

// Modelled duration of a matvec launch over nt tiles of 256 targets and nt of 256 sources in
// ns source slices on a device of ncu compute units. The kernel is bound by instruction issue,
// which a compute unit shares among its resident workgroups, so each unit is modelled as
// working through the workgroups it is given one after another: workgroups go out in
// dispatch order (target block fastest) to the unit that frees up first, each taking its
// slice's tile count plus half a tile (loading its targets, writing its partial sums).
double matvec_makespan(int64_t nt, int64_t ns, int64_t ncu) {
  const int64_t L = (nt + ns - 1) / ns;
  std::priority_queue<double, std::vector<double>, std::greater<double>> busy;  // finish times
  double end = 0.0;
  for (int64_t y = 0; y < ns; ++y) {
    const double d = (double)std::max<int64_t>(0, std::min(L, nt - y * L)) + 0.5;
    for (int64_t x = 0; x < nt; ++x) {
      double start = 0.0;
      if ((int64_t)busy.size() >= ncu) {
        start = busy.top();
        busy.pop();
      }
      busy.push(start + d);
      end = std::max(end, start + d);
    }
  }
  return end;
}

}  // namespace

int matvec_slices(int64_t n, int64_t max_entries) {
  if (n <= 0) return 1;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(kMatvecMaxSlices, max_entries / n));
  int dev = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::tuple<int, int64_t, int64_t>, int> memo;
  const auto key = std::make_tuple(dev, n, cap);
  {
    std::lock_guard<std::mutex> l(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  // at least seven workgroups per compute unit (enough resident waves to keep issue busy),
  // then the fewest slices whose modelled duration is within 2% of the best
  int ncu = 0;
  FMMLU_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  ncu = std::max(ncu, 1);
  const int64_t nt = (n + 255) / 256;
  const int64_t smin = std::min(cap, std::max<int64_t>(1, (7 * (int64_t)ncu + nt - 1) / nt));
  std::vector<double> t((size_t)cap + 1, 0.0);
  double best = -1.0;
  for (int64_t s = smin; s <= cap; ++s) {
    t[(size_t)s] = matvec_makespan(nt, s, ncu);
    best = best < 0.0 ? t[(size_t)s] : std::min(best, t[(size_t)s]);
  }
  int ns = (int)smin;
  while (t[(size_t)ns] > best * 1.02) ++ns;
  std::lock_guard<std::mutex> l(mu);
  memo[key] = ns;
  return ns;
}

void launch_matvec(const DevGeom& g, int op, const zd* x, zd* y, zd* part, int64_t part_entries,
                   hipStream_t st) {
  if (g.n <= 0) return;
  const int ns = matvec_slices(g.n, part_entries);
  if ((int64_t)ns * g.n > part_entries) throw Error(FMMLU_EINVAL, "internal: matvec partials exceed their buffer");
  const int64_t nt = (g.n + 255) / 256;
  const int64_t slice = (nt + ns - 1) / ns * 256;
  const dim3 grid((unsigned)nt, (unsigned)ns), b(256);
  const bool fast = g.kr_max < kPhaseFast;
#define FMMLU_MATVEC_LAUNCH(OPV)                                                              \
  do {                                                                                        \
    if (fast)                                                                                 \
      hipLaunchKernelGGL((matvec_kernel<OPV, true>), grid, b, 0, st, g, x, part, slice);     \
    else                                                                                      \
      hipLaunchKernelGGL((matvec_kernel<OPV, false>), grid, b, 0, st, g, x, part, slice);    \
  } while (0)
  if (op == 0)
    FMMLU_MATVEC_LAUNCH(0);
  else if (op == 1)
    FMMLU_MATVEC_LAUNCH(1);
  else if (op == 2)
    FMMLU_MATVEC_LAUNCH(2);
  else
    FMMLU_MATVEC_LAUNCH(3);
#undef FMMLU_MATVEC_LAUNCH
  FMMLU_HIP(hipGetLastError());
  hipLaunchKernelGGL(matvec_sum_kernel, dim3((unsigned)((g.n + 255) / 256)), b, 0, st, part, g.n, ns, y);
  FMMLU_HIP(hipGetLastError());
  if (g.corr.rptr) {
    const dim3 gc((unsigned)((g.n + 255) / 256));
    if (op == 0)
      hipLaunchKernelGGL(matvec_corr_kernel<0>, gc, b, 0, st, g, x, y);
    else if (op == 1)
      hipLaunchKernelGGL(matvec_corr_kernel<1>, gc, b, 0, st, g, x, y);
    else if (op == 2)
      hipLaunchKernelGGL(matvec_corr_kernel<2>, gc, b, 0, st, g, x, y);
    else
      hipLaunchKernelGGL(matvec_corr_kernel<3>, gc, b, 0, st, g, x, y);
    FMMLU_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------------------------------
// Scratch of the allocation-free matvec: a file-scope device array, one copy per GPU, held
// until the process ends. Host code never names it directly: its device address on each GPU
// comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) zd scratch[kNoallocScratchBytes / sizeof(zd)];

int64_t matvec_noalloc_part_entries(int64_t n) { return (int64_t)(kNoallocScratchBytes / sizeof(zd)) - 2 * n; }

int64_t matvec_noalloc_entries(int64_t n) {
  return (2 + (int64_t)matvec_slices(n, matvec_noalloc_part_entries(n))) * n;
}

zd* noalloc_scratch() {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static zd* ptr[kMaxDev] = {};
  int dev = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) throw Error(FMMLU_EINVAL, "device ordinal " + std::to_string(dev) + " out of range");
  std::lock_guard<std::mutex> l(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    FMMLU_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(FMMLU_EHIP, "hipGetSymbolAddress returned a null address for the matvec scratch");
    ptr[dev] = static_cast<zd*>(p);
  }
  return ptr[dev];
}

}  // namespace fmmlu
