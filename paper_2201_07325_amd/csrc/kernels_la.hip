// Batched dense linear algebra on complex float64 for uneven sizes: GEMM with segments and
// scatter maps, Householder panel QR (compact WY), greedy column-pivoted QR on a square
// factor, Gauss-Jordan inversion with partial pivoting, and block gathers.
//
// All matrices are column-major. Workgroups are 256 threads (four 64-wide wavefronts);
// reductions go through wavefront shuffles first and LDS second.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

#include <atomic>
#include <mutex>

namespace fmmlu {

namespace {

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

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of a complex value over the 256-thread block; result broadcast to all threads.
__device__ inline zd block_sum(zd v, zd* red /* >= 4 */) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  zd s = red[0];
  for (int i = 1; i < 4; ++i) s = zadd(s, red[i]);
  __syncthreads();
  return s;
}

__device__ inline double block_sum_d(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------------------
// Householder QR of the panel A[j0:rows, j0:j0+nb], nb <= kQrNb. Reflector H = I - tau v v^H
// with v = x + e^{i arg x0} |x| e_1 and tau = 2/|v|^2 (Hermitian, unitary), so that
// H x = -e^{i arg x0} |x| e_1. The product H_1 ... H_nb = I - V Tw V^H (compact WY, forward)
// is returned with V written explicitly. One workgroup per panel; per column two passes over
// the panel rows (dots, then update + next column's norm), each closed by one reduction.
constexpr int kQrNb = 16;

template <int N>
__device__ inline void block_reduce_vec(zd (&v)[N], zd (*red)[N], zd* out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double re = wave_sum(v[q].re), im = wave_sum(v[q].im);
    if (lane == 0) red[w][q] = zd{re, im};
  }
  __syncthreads();
  if (threadIdx.x < N) {
    zd a = red[0][threadIdx.x];
    for (int i = 1; i < 4; ++i) a = zadd(a, red[i][threadIdx.x]);
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) qr_panel_kernel(const QrTask* __restrict__ tasks) {
  constexpr int NB = kQrNb;
  const QrTask t = tasks[blockIdx.x];
  __shared__ zd red[4][2 * NB];
  __shared__ zd s_d[2 * NB];
  __shared__ double redd[4];
  __shared__ double s_ss;
  __shared__ zd s_v0, s_beta;
  __shared__ double s_tau;
  const int L = t.rows - t.j0;  // panel height
  const int nb = t.nb;
  const int64_t lda = t.lda;
  zd* P = t.A + t.j0 + (int64_t)t.j0 * lda;  // P[i + c*lda], i < L, c < nb
  zd* V = t.V;
  const int64_t ldv = L;
  for (int e = threadIdx.x; e < nb * nb; e += 256) t.Tw[e] = zd{0.0, 0.0};
  double ss = 0.0;
  for (int i = threadIdx.x; i < L; i += 256) ss += zabs2(P[i]);
  ss = block_sum_d(ss, redd);
  if (threadIdx.x == 0) s_ss = ss;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (j >= L) {
      for (int i = threadIdx.x; i < L; i += 256) V[i + j * ldv] = zd{0.0, 0.0};
      continue;
    }
    if (threadIdx.x == 0) {
      const zd a = P[j + (int64_t)j * lda];
      const double nrm = sqrt(s_ss);
      const double aa = sqrt(zabs2(a));
      const zd ph = aa > 0.0 ? zd{a.re / aa, a.im / aa} : zd{1.0, 0.0};
      const zd v0 = zd{a.re + ph.re * nrm, a.im + ph.im * nrm};
      const double vn2 = s_ss - zabs2(a) + zabs2(v0);
      s_v0 = v0;
      s_tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      s_beta = zd{-ph.re * nrm, -ph.im * nrm};
    }
    __syncthreads();
    const zd v0 = s_v0;
    const double tau = s_tau;
    // pass A: d_c = v^H P[:, c] (c > j) and w_l = V_l^H v (l < j)
    zd acc[2 * NB];
#pragma unroll
    for (int q = 0; q < 2 * NB; ++q) acc[q] = zd{0.0, 0.0};
    for (int i = j + threadIdx.x; i < L; i += 256) {
      const zd vi = (i == j) ? v0 : P[i + (int64_t)j * lda];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c > j && c < nb) zfmac(acc[c], vi, P[i + (int64_t)c * lda]);
#pragma unroll
      for (int l = 0; l < NB; ++l)
        if (l < j) zfmac(acc[NB + l], V[i + l * ldv], vi);
    }
    block_reduce_vec<2 * NB>(acc, red, s_d);
    // pass B: update columns c > j; V column j; R column j; norm^2 of column j+1 below row j+1
    double ss2 = 0.0;
    for (int i = threadIdx.x; i < L; i += 256) {
      if (i < j) {
        V[i + j * ldv] = zd{0.0, 0.0};
        continue;
      }
      const zd vi = (i == j) ? v0 : P[i + (int64_t)j * lda];
      V[i + j * ldv] = vi;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c > j && c < nb) {
          zd* pc = P + i + (int64_t)c * lda;
          const zd f = zscale(zmul(vi, s_d[c]), tau);
          const zd nv = zsub(*pc, f);
          *pc = nv;
          if (c == j + 1 && i >= j + 1) ss2 += zabs2(nv);
        }
      }
      P[i + (int64_t)j * lda] = (i == j) ? s_beta : zd{0.0, 0.0};
    }
    ss2 = block_sum_d(ss2, redd);
    if (threadIdx.x == 0) {
      s_ss = ss2;
      for (int r = 0; r < j; ++r) {
        zd sacc{0.0, 0.0};
        for (int l = r; l < j; ++l) zfma(sacc, t.Tw[r + l * nb], s_d[NB + l]);
        t.Tw[r + j * nb] = zscale(sacc, -tau);
      }
      t.Tw[j + j * nb] = zd{tau, 0.0};
    }
    __syncthreads();
  }
}

// Split-K partial sums of W = V^H A2 are reduced and multiplied by Tw^H in one pass:
// W2[:, c] = Tw^H sum_k part_k[:, c]. One thread per column.
__global__ void __launch_bounds__(256) reduce_tw_kernel(const RedTwTask* __restrict__ tasks) {
  const RedTwTask t = tasks[blockIdx.x];
  const int c = blockIdx.y * 256 + threadIdx.x;
  if (c >= t.ncols) return;
  zd w[kQrNb];
  for (int q = 0; q < t.nb; ++q) w[q] = zd{0.0, 0.0};
  for (int k = 0; k < t.nsplit; ++k) {
    const zd* p = t.part + (int64_t)k * t.part_stride + (int64_t)c * t.nb;
    for (int q = 0; q < t.nb; ++q) w[q] = zadd(w[q], p[q]);
  }
  zd* o = t.W2 + (int64_t)c * t.nb;
  for (int r = 0; r < t.nb; ++r) {
    // (Tw^H w)_r = sum_q conj(Tw[q, r]) w_q, Tw upper triangular (q <= r)
    zd a{0.0, 0.0};
    for (int q = 0; q <= r; ++q) zfmac(a, t.Tw[q + r * t.nb], w[q]);
    o[r] = a;
  }
}

// ---------------------------------------------------------------------------------------
// T = R11^{-1} R12 for R (m x m, ld lda) with rank s: T is s x (m - s), written with ld m.
// The right-hand sides are processed transposed in scratch W (W[c + i*nc], nc = m - s) so
// that the lanes of a wavefront, one right-hand side each, touch consecutive addresses;
// R's column i is read as a broadcast. Call from all 256 threads after a barrier.
template <int NT>
__device__ inline void back_substitute_n(const zd* __restrict__ R, int64_t lda, int s, int m, zd* W,
                                         zd* T, bool real_diag) {
  const int nc = m - s;
  for (int e = threadIdx.x; e < s * nc; e += NT) {
    const int c = e % nc, i = e / nc;
    W[c + (int64_t)i * nc] = R[i + (int64_t)(s + c) * lda];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += NT) {
    for (int i = s - 1; i >= 0; --i) {
      const zd rii = R[i + (int64_t)i * lda];
      const zd ti = real_diag ? zscale(W[c + (int64_t)i * nc], 1.0 / rii.re) : zdiv(W[c + (int64_t)i * nc], rii);
      W[c + (int64_t)i * nc] = ti;
      const zd* ri = R + (int64_t)i * lda;
      for (int r = 0; r < i; ++r) W[c + (int64_t)r * nc] = zsub(W[c + (int64_t)r * nc], zmul(ri[r], ti));
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * nc; e += NT) {
    const int i = e % s, c = e / s;
    T[i + (int64_t)c * m] = W[c + (int64_t)i * nc];
  }
}
__device__ inline void back_substitute(const zd* __restrict__ R, int64_t lda, int s, int m, zd* W,
                                       zd* T, bool real_diag) {
  back_substitute_n<256>(R, lda, s, m, W, T, real_diag);
}

// ---------------------------------------------------------------------------------------
// Greedy CPQR of an m x m matrix in place, then T = R11^{-1} R12 (ld m). The squared norms
// of the trailing columns are recomputed exactly at every step, fused into the reflector
// pass (dynamic LDS holds them: m doubles). Ties go to the lowest original column index.
__global__ void __launch_bounds__(256) cpqr_kernel(const CpqrTask* __restrict__ tasks, double eps) {
  const CpqrTask t = tasks[blockIdx.x];
  const int m = t.m;
  const int64_t lda = t.lda;
  zd* R = t.R;
  extern __shared__ double nrm2[];
  __shared__ double bestv[4];
  __shared__ int besti[4];
  __shared__ int bestp[4];
  __shared__ int sh_piv, sh_stop;
  __shared__ double sh_r00;
  __shared__ zd sh_v0, sh_beta;
  __shared__ double sh_tau;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = threadIdx.x; j < m; j += 256) t.perm[j] = j;
  for (int c = wave; c < m; c += 4) {
    double acc = 0.0;
    const zd* col = R + (int64_t)c * lda;
    for (int i = lane; i < m; i += 64) acc += zabs2(col[i]);
    acc = wave_sum(acc);
    if (lane == 0) nrm2[c] = acc;
  }
  __syncthreads();
  int s = m;
  for (int k = 0; k < m; ++k) {
    // argmax of nrm2[k..m), ties -> lowest original index
    double mb = -1.0;
    int mi = -1, mp = 0x7fffffff;
    for (int c = k + threadIdx.x; c < m; c += 256) {
      const double v = nrm2[c];
      const int pc = t.perm[c];
      if (v > mb || (v == mb && pc < mp)) {
        mb = v;
        mi = c;
        mp = pc;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(mb, o, 64);
      const int oi = __shfl_xor(mi, o, 64);
      const int op = __shfl_xor(mp, o, 64);
      if (oi >= 0 && (mi < 0 || ov > mb || (ov == mb && op < mp))) {
        mb = ov;
        mi = oi;
        mp = op;
      }
    }
    if (lane == 0) {
      bestv[wave] = mb;
      besti[wave] = mi;
      bestp[wave] = mp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = -1.0;
      int bi = -1, bp = 0x7fffffff;
      for (int w = 0; w < 4; ++w) {
        if (besti[w] < 0) continue;
        if (bi < 0 || bestv[w] > bv || (bestv[w] == bv && bestp[w] < bp)) {
          bv = bestv[w];
          bi = besti[w];
          bp = bestp[w];
        }
      }
      const double nk = sqrt(fmax(bv, 0.0));
      int stop = 0;
      if (k == 0) {
        sh_r00 = nk;
        if (nk == 0.0) stop = 1;
      } else if (nk <= eps * sh_r00) {
        stop = 1;
      }
      sh_stop = stop;
      sh_piv = bi;
    }
    __syncthreads();
    if (sh_stop) {
      s = k;
      break;
    }
    const int p = sh_piv;
    if (p != k) {
      for (int i = threadIdx.x; i < m; i += 256) {
        zd a = R[i + (int64_t)k * lda];
        R[i + (int64_t)k * lda] = R[i + (int64_t)p * lda];
        R[i + (int64_t)p * lda] = a;
      }
      if (threadIdx.x == 0) {
        int q = t.perm[k];
        t.perm[k] = t.perm[p];
        t.perm[p] = q;
        double d = nrm2[k];
        nrm2[k] = nrm2[p];
        nrm2[p] = d;
      }
    }
    __syncthreads();
    zd* x = R + k + (int64_t)k * lda;
    const int len = m - k;
    if (threadIdx.x == 0) {
      const double ss = nrm2[k];
      const zd a = x[0];
      const double nrm = sqrt(ss);
      const double aa = sqrt(zabs2(a));
      const zd ph = aa > 0.0 ? zd{a.re / aa, a.im / aa} : zd{1.0, 0.0};
      const zd v0 = zd{a.re + ph.re * nrm, a.im + ph.im * nrm};
      const double vn2 = ss - zabs2(a) + zabs2(v0);
      sh_v0 = v0;
      sh_tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      sh_beta = zd{-ph.re * nrm, -ph.im * nrm};
    }
    __syncthreads();
    const zd v0 = sh_v0;
    const double tau = sh_tau;
    // apply to columns k+1..m-1 (wave per column); new squared norm below row k
    for (int c = k + 1 + wave; c < m; c += 4) {
      zd* col = R + k + (int64_t)c * lda;
      zd d{0.0, 0.0};
      for (int i = lane; i < len; i += 64) zfmac(d, (i == 0) ? v0 : x[i], col[i]);
      d.re = wave_sum(d.re);
      d.im = wave_sum(d.im);
      const zd f = zscale(d, tau);
      double nn = 0.0;
      for (int i = lane; i < len; i += 64) {
        const zd nv = zsub(col[i], zmul((i == 0) ? v0 : x[i], f));
        col[i] = nv;
        if (i > 0) nn += zabs2(nv);
      }
      nn = wave_sum(nn);
      if (lane == 0) nrm2[c] = nn;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 256) x[i] = (i == 0) ? sh_beta : zd{0.0, 0.0};
    __syncthreads();
  }
  if (threadIdx.x == 0) *t.rank = s;
  __syncthreads();
  back_substitute(R, lda, s, m, t.W, t.T, false);
}

// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) sum_parts_kernel(const SumTask* __restrict__ tasks, int ntasks) {
  const int64_t u = blockIdx.x;
  const int ti = find_task(tasks, ntasks, u);
  const SumTask t = tasks[ti];
  const int64_t e = (u - t.unit_begin) * 256 + threadIdx.x;
  if (e >= t.count) return;
  int64_t i = 0, j = 0;
  if (t.herm > 0) {
    i = e % t.herm;
    j = e / t.herm;
    if (i < j) return;
  }
  zd a{0.0, 0.0};
  for (int k = 0; k < t.nsplit; ++k) a = zadd(a, t.part[(int64_t)k * t.stride + e]);
  t.out[e] = a;
  if (t.herm > 0 && i > j) t.out[j + i * t.herm] = zconj(a);
}

// Left-looking pivoted Cholesky of the Gram matrix (greedy CPQR of M in exact arithmetic).
// Row k of R is R[k, c] = (G[p_k, c] - sum_{l<k} conj(R[l, p_k]) R[l, c]) / R[k, k] for every
// column c not yet chosen, p_k maximising the Schur-complement diagonal dg (the squared norm
// of column c of M after projection on the chosen columns; ties to the lowest column). R is
// kept row-major by original column (Rt[l m + c]), so the sum is one coalesced pass over the
// previous rows (split into row slices when m is small). G is stored with both triangles, so
// row p_k is read as the contiguous column, G[p_k, c] = conj(G[c, p_k]). Positions follow
// column-pivoted QR's exchange rule (step k swaps positions
// k and pos(p_k)). At the end R is written in pivoted column order, column-major (rows < rank,
// upper triangle only), for the back substitution.
// (value, index) ordering of pivot searches: larger value, ties to the smaller index
__device__ inline bool gj_better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// 32-bit lane permutation of a wave (DPP) applied to a double and an int
template <int CTRL>
__device__ inline void gj_dpp(double& v, int& i) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  const int ii = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  const double ov = __hiloint2double(hi, lo);
  if (gj_better(ov, ii, v, i)) {
    v = ov;
    i = ii;
  }
}

// (value, row) with the largest value, ties to the smaller row, in every lane of the wave:
// quads (DPP quad_perm), half rows and rows of 16 (DPP mirrors), then across rows.
__device__ inline void gj_wave_argmax(double& v, int& i) {
  gj_dpp<0xB1>(v, i);   // quad_perm [1,0,3,2]
  gj_dpp<0x4E>(v, i);   // quad_perm [2,3,0,1]
  gj_dpp<0x141>(v, i);  // row_half_mirror
  gj_dpp<0x140>(v, i);  // row_mirror
  for (int o = 16; o <= 32; o <<= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(i, o, 64);
    if (gj_better(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
}

constexpr int kPcholThreads = 1024;

// rank, perm = pv, and the rows < s of R in pivoted order (column-major, ld m, upper
// triangle) through a 32 x 32 LDS tile (part: >= 32 x 33 entries): reads along rows of Rt,
// writes down columns. Called by all NT threads.
template <int NT>
__device__ inline void pchol_write_out(const PcholTask& t, int s, const int* pv, zd* part, int ib = 0,
                                       int nib = 1, bool stopped = true) {
  const int m = t.m, tid = threadIdx.x;
  const zd* __restrict__ Rt = t.Rt;
  if (ib == 0) {
    if (tid == 0) *t.rank = stopped ? s : -1 - s;
    for (int j = tid; j < m; j += NT) t.perm[j] = pv[j];
  }
  zd(*tile)[33] = reinterpret_cast<zd(*)[33]>(part);
  for (int i0 = 32 * ib; i0 < s; i0 += 32 * nib) {
    for (int j0 = i0 & ~31; j0 < m; j0 += 32) {
      __syncthreads();
      for (int e = tid; e < 1024; e += NT) {
        const int ta = e & 31, tb = e >> 5;
        const int i = i0 + tb, j = j0 + ta;
        zd v{0.0, 0.0};
        if (i < s && j < m && j >= i) v = Rt[(int64_t)i * m + pv[j]];
        tile[tb][ta] = v;
      }
      __syncthreads();
      for (int e = tid; e < 1024; e += NT) {
        const int ta = e & 31, tb = e >> 5;
        const int i = i0 + ta, j = j0 + tb;
        if (i < s && j < m) t.Rp[i + (int64_t)j * m] = tile[ta][tb];
      }
    }
  }
}

// G[p, c] of the Hermitian G (column-major, ld m, both triangles): column p, conjugated
__device__ inline zd pchol_grow(const zd* __restrict__ G, int m, int p, int c) {
  return zconj(G[c + (int64_t)p * m]);
}

__device__ inline bool pchol_better(double v, int c, double bv, int bc) {
  return c >= 0 && (bc < 0 || v > bv || (v == bv && c < bc));
}

template <int NT>
__global__ void __launch_bounds__(NT) pchol_kernel(const PcholTask* __restrict__ tasks, double eps, int mult_in_lds) {
  const PcholTask t = tasks[blockIdx.x];
  const int m = t.m;
  const zd* __restrict__ G = t.G;
  zd* __restrict__ Rt = t.Rt;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ zd part[32 * 33];  // row-slice partial sums; 32 x 33 tile in the final pass
  __shared__ double bestv[NT / 64];
  __shared__ int bestc[NT / 64];
  zd* mult = mult_in_lds ? reinterpret_cast<zd*>(smem) : t.Rp;  // R[0:k, p_k]
  double* dg = reinterpret_cast<double*>(smem + (mult_in_lds ? sizeof(zd) * (size_t)m : 0));
  int* pos = reinterpret_cast<int*>(dg + m);  // column -> position
  int* pv = pos + m;                          // position -> column
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int c = tid; c < m; c += NT) {
    dg[c] = G[c + (int64_t)c * m].re;
    pos[c] = c;
    pv[c] = c;
  }
  __syncthreads();
  const int mpad = (m + 63) & ~63;
  const int slices = mpad >= NT ? 1 : NT / mpad;
  double r00 = 0.0;
  int s = m;
  for (int k = 0; k < m; ++k) {
    double bv = -1.0;
    int bc = -1;
    for (int c = tid; c < m; c += NT) {
      if (pos[c] < k) continue;
      const double v = dg[c];
      if (pchol_better(v, c, bv, bc)) {
        bv = v;
        bc = c;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oc = __shfl_xor(bc, o, 64);
      if (pchol_better(ov, oc, bv, bc)) {
        bv = ov;
        bc = oc;
      }
    }
    if (lane == 0) {
      bestv[wave] = bv;
      bestc[wave] = bc;
    }
    __syncthreads();
    bv = -1.0;
    bc = -1;
    for (int w = 0; w < NT / 64; ++w)
      if (pchol_better(bestv[w], bestc[w], bv, bc)) {
        bv = bestv[w];
        bc = bestc[w];
      }
    const int p = bc;
    const double rkk = sqrt(fmax(bv, 0.0));
    if (k == 0) r00 = rkk;
    if (p < 0 || (k == 0 ? rkk == 0.0 : rkk <= eps * r00)) {
      s = k;
      break;
    }
    if (tid == 0) {
      const int q = pos[p], ck = pv[k];
      pv[k] = p;
      pv[q] = ck;
      pos[p] = k;
      pos[ck] = q;
    }
    for (int l = tid; l < k; l += NT) mult[l] = Rt[(int64_t)l * m + p];
    __syncthreads();
    const double inv = 1.0 / rkk;
    if (slices == 1) {
      for (int c = tid; c < m; c += NT) {
        if (pos[c] <= k) continue;
        zd a0{0.0, 0.0}, a1{0.0, 0.0};
        int l = 0;
        for (; l + 1 < k; l += 2) {
          zfmac(a0, mult[l], Rt[(int64_t)l * m + c]);
          zfmac(a1, mult[l + 1], Rt[(int64_t)(l + 1) * m + c]);
        }
        if (l < k) zfmac(a0, mult[l], Rt[(int64_t)l * m + c]);
        const zd v = zscale(zsub(pchol_grow(G, m, p, c), zadd(a0, a1)), inv);
        Rt[(int64_t)k * m + c] = v;
        dg[c] -= zabs2(v);
      }
    } else {
      const int q = tid / mpad, c = tid - q * mpad;
      zd acc{0.0, 0.0};
      if (q < slices && c < m && pos[c] > k) {
        const int L = (k + slices - 1) / slices;
        const int l0 = q * L, l1 = min(k, l0 + L);
        for (int l = l0; l < l1; ++l) zfmac(acc, mult[l], Rt[(int64_t)l * m + c]);
      }
      if (q < slices) part[tid] = acc;
      __syncthreads();
      if (tid < m && pos[tid] > k) {
        zd sum = part[tid];
        for (int qq = 1; qq < slices; ++qq) sum = zadd(sum, part[qq * mpad + tid]);
        const zd v = zscale(zsub(pchol_grow(G, m, p, tid), sum), inv);
        Rt[(int64_t)k * m + tid] = v;
        dg[tid] -= zabs2(v);
      }
    }
    if (tid == 0) Rt[(int64_t)k * m + p] = zd{rkk, 0.0};
    __syncthreads();
  }
  pchol_write_out<NT>(t, s, pv, part);
}

// One block of kPcholNb pivots of the blocked pivoted Cholesky (see PcholTask): G holds the
// Schur complement of the Gram matrix after the earlier blocks (both triangles), so row k of
// R is R[k, c] = (G[p_k, c] - sum_{k0 <= l < k} conj(R[l, p_k]) R[l, c]) / R[k, k]. Thread c
// keeps column c's rows of the block in registers; the pivot column's values are broadcast
// through LDS. State (dg, positions, k, done) lives in global memory between launches.
template <int NT>
__global__ void __launch_bounds__(NT) pchol_block_kernel(const PcholTask* __restrict__ tasks, int k0, double eps) {
  constexpr int NB = kPcholNb, NW = NT / 64;
  const PcholTask t = tasks[blockIdx.x];
  const int m = t.m;
  if (k0 >= m) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* dgs = t.dgs;
  int* gpos = t.ist;
  int* gpv = t.ist + m;
  int* ctl = t.ist + 2 * m;  // [0] k reached, [1] done
  __shared__ int pos[NT], pv[NT];
  __shared__ double bestv[NW];
  __shared__ int bestc[NW];
  __shared__ zd multb[NB];
  __shared__ int sh_done, sh_p;
  __shared__ double sh_r00;
  if (k0 == 0) {
    for (int c = tid; c < m; c += NT) {
      dgs[c] = t.G[c + (int64_t)c * m].re;
      pos[c] = c;
      pv[c] = c;
    }
    if (tid == 0) {
      ctl[0] = 0;
      ctl[1] = 0;
      dgs[m] = 0.0;
    }
  } else {
    for (int c = tid; c < m; c += NT) {
      pos[c] = gpos[c];
      pv[c] = gpv[c];
    }
  }
  __syncthreads();
  if (tid == 0) {
    sh_done = ctl[1];
    sh_r00 = dgs[m];
  }
  __syncthreads();
  const int c = tid;  // this thread's column (m <= NT)
  zd rb[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) rb[j] = zd{0.0, 0.0};
  double dgc = c < m ? dgs[c] : 0.0;
  if (!sh_done) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = k0 + j;
      if (k >= m || sh_done) break;
      // pivot: the remaining column with the largest Schur-complement diagonal (ties: lowest)
      // non-candidates carry (-inf, m): every candidate beats them, and their ties stay
      double bv = -INFINITY;
      int bc = m;
      if (c < m && pos[c] >= k) {
        bv = dgc;
        bc = c;
      }
      gj_wave_argmax(bv, bc);
      if (lane == 0) {
        bestv[wave] = bv;
        bestc[wave] = bc;
      }
      __syncthreads();
      bv = bestv[0];
      bc = bestc[0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (gj_better(bestv[w], bestc[w], bv, bc)) {
          bv = bestv[w];
          bc = bestc[w];
        }
      if (bc >= m) bc = -1;  // no candidate left
      const int p = bc;
      const double rkk = sqrt(fmax(bv, 0.0));
      const double r00 = k == 0 ? rkk : sh_r00;
      const bool stop = p < 0 || (k == 0 ? rkk == 0.0 : rkk <= eps * r00);
      if (stop) {
        if (tid == 0) {
          sh_done = 1;
          ctl[1] = 1;
          ctl[0] = k;
        }
        __syncthreads();
        break;
      }
      if (tid == 0) {
        if (k == 0) sh_r00 = rkk;
        const int q = pos[p], ck = pv[k];
        pv[k] = p;
        pv[q] = ck;
        pos[p] = k;
        pos[ck] = q;
        sh_p = p;
      }
      if (c == p) {
#pragma unroll
        for (int l = 0; l < NB; ++l)
          if (l < j) multb[l] = rb[l];
      }
      __syncthreads();
      const double inv = 1.0 / rkk;
      if (c < m) {
        if (c == p) {
          rb[j] = zd{rkk, 0.0};
          t.Rt[(int64_t)k * m + c] = rb[j];
        } else if (pos[c] > k) {
          zd acc{0.0, 0.0};
#pragma unroll
          for (int l = 0; l < NB; ++l)
            if (l < j) zfmac(acc, multb[l], rb[l]);
          const zd g = pchol_grow(t.G, m, p, c);
          const zd v = zscale(zsub(g, acc), inv);
          rb[j] = v;
          t.Rt[(int64_t)k * m + c] = v;
          dgc -= zabs2(v);
        }
      }
      __syncthreads();
    }
  }
  // the block's rows for the downdate (zero where nothing was computed), and the state
  if (c < m) {
#pragma unroll
    for (int j = 0; j < NB; ++j) t.Rb[j + (int64_t)c * NB] = rb[j];
    dgs[c] = dgc;
    gpos[c] = pos[c];
    gpv[c] = pv[c];
  }
  if (tid == 0) {
    dgs[m] = sh_r00;
    if (!sh_done) ctl[0] = min(m, k0 + NB);
    if (!sh_done && k0 + NB >= m) ctl[1] = 1;
  }
}

// after the last block: rank, perm and R in pivoted order
// one workgroup per (box, 32-row block of R): blocks at or past the rank have nothing to write.
// A box whose pivoting has not stopped yet (the blocks launched so far did not reach its
// rank) gets rank -1 - (pivots so far); the caller launches the remaining blocks and this
// kernel again.
__global__ void __launch_bounds__(kPcholThreads) pchol_finish_kernel(const PcholTask* __restrict__ tasks) {
  const PcholTask t = tasks[blockIdx.x];
  const int s = t.ist[2 * t.m];
  const bool stopped = t.ist[2 * t.m + 1] != 0;
  if (blockIdx.y > 0 && 32 * (int)blockIdx.y >= s) return;
  __shared__ zd part[32 * 33];
  extern __shared__ int pvs[];
  for (int j = threadIdx.x; j < t.m; j += kPcholThreads) pvs[j] = t.ist[t.m + j];
  __syncthreads();
  pchol_write_out<kPcholThreads>(t, s, pvs, part, (int)blockIdx.y, (int)gridDim.y, stopped);
}

// T = R11^{-1} R12 (s x (m - s), ld m) from R in pivoted order. Each workgroup holds NC
// right-hand-side columns in LDS; blocks of 16 rows are solved there (diagonal block staged
// in LDS, one thread per column), then the rows above are updated in one pass over the
// block's 16 columns of R.
template <int NC>
__global__ void __launch_bounds__(256) pchol_t_kernel(const PcholTask* __restrict__ tasks) {
  const PcholTask t = tasks[blockIdx.x];
  const int m = t.m, s = *t.rank;
  const int c0 = blockIdx.y * NC;
  if (s <= 0 || c0 >= m - s) return;  // s < 0: pivoting not finished (see pchol_finish_kernel)
  const int nc = min(NC, m - s - c0);
  extern __shared__ __align__(16) unsigned char smem[];
  zd* W = reinterpret_cast<zd*>(smem);  // W[i * NC + j], i < s
  __shared__ zd Rb[16][17];
  __shared__ double dinv[16];
  const zd* __restrict__ Rp = t.Rp;
  const int tid = threadIdx.x;
  for (int e = tid; e < s * NC; e += 256) {
    const int i = e % s, j = e / s;
    W[i * NC + j] = j < nc ? Rp[i + (int64_t)(s + c0 + j) * m] : zd{0.0, 0.0};
  }
  for (int i1 = s; i1 > 0; i1 -= 16) {
    const int i0 = max(0, i1 - 16), b = i1 - i0;
    __syncthreads();
    {
      const int r = tid & 15, c = tid >> 4;
      if (r < b && c < b && r <= c) Rb[r][c] = Rp[(i0 + r) + (int64_t)(i0 + c) * m];
      if (tid < b) dinv[tid] = 1.0 / Rp[(i0 + tid) + (int64_t)(i0 + tid) * m].re;
    }
    __syncthreads();
    // the diagonal block: one thread per right-hand-side column, in registers (the same
    // operations in the same order as a row-by-row sweep, without a barrier per row)
    if (tid < NC) {
      zd w[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) w[q] = q < b ? W[(i0 + q) * NC + tid] : zd{0.0, 0.0};
#pragma unroll
      for (int i = 15; i >= 0; --i) {
        if (i < b) {
          w[i] = zscale(w[i], dinv[i]);
#pragma unroll
          for (int r = 0; r < i; ++r) w[r] = zsub(w[r], zmul(Rb[r][i], w[i]));
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < b) W[(i0 + q) * NC + tid] = w[q];
    }
    __syncthreads();
    for (int r = tid; r < i0; r += 256) {
      zd a[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = q < b ? Rp[r + (int64_t)(i0 + q) * m] : zd{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        zd acc = W[r * NC + j];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < b) acc = zsub(acc, zmul(a[q], W[(i0 + q) * NC + j]));
        W[r * NC + j] = acc;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < s * nc; e += 256) {
    const int i = e % s, j = e / s;
    t.T[i + (int64_t)(c0 + j) * m] = W[i * NC + j];
  }
}

// ---------------------------------------------------------------------------------------
// Gauss-Jordan inversion with partial pivoting, blocked by column panels of kGjNb.
constexpr int kGjNb = kGjBlock;

// Panel: columns J = [j0, j0+nb) of all n rows; pivot rows searched among rows >= column
// (largest modulus, ties to the lowest row). Each thread keeps one row of the panel in
// registers for all nb steps. A matrix taller than one workgroup is split over wpt
// workgroups that meet once per column: each publishes its best candidate row (and the
// owner of the pivot position publishes that row) in a double-buffered slot, arrives at a
// counter, and waits (bounded) until all have arrived; the pivot row then comes from the
// winning slot. Launched cooperatively, so all workgroups are resident.
constexpr int64_t kGjSpinLimit = int64_t(1) << 22;


__global__ void __launch_bounds__(256) gj_panel_kernel(const GjTask* __restrict__ tasks, int j0) {
  const GjTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (j0 >= n) return;
  const int w = blockIdx.y;
  if (w >= t.wpt) return;
  const int nb = min(kGjNb, n - j0);
  const int64_t lda = t.lda;
  zd* A = t.A;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int gi = w * kGjPanelRows + tid;
  const bool own = gi < n;
  __shared__ double bv[4];
  __shared__ int bi[4];
  __shared__ zd prow[kGjNb], rowgc[kGjNb];
  __shared__ int sh_win, sh_p;
  __shared__ double sh_best;
  zd a[kGjNb];
#pragma unroll
  for (int q = 0; q < kGjNb; ++q) a[q] = (own && q < nb) ? A[gi + (int64_t)(j0 + q) * lda] : zd{0.0, 0.0};
  const bool multi = t.wpt > 1;
  const int64_t slen = gj_slot_len(t.wpt);
  for (int j = 0; j < kGjNb; ++j) {
    if (j < nb) {
      const int gc = j0 + j;
      zd aj = a[0];
#pragma unroll
      for (int q = 1; q < kGjNb; ++q)
        if (q == j) aj = a[q];
      double best = -1.0;
      int besti = 0x7fffffff;
      if (own && gi >= gc) {
        best = zabs2(aj);
        besti = gi;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(besti, o, 64);
        if (gj_better(ov, oi, best, besti)) {
          best = ov;
          besti = oi;
        }
      }
      if (lane == 0) {
        bv[wave] = best;
        bi[wave] = besti;
      }
      __syncthreads();
      if (tid == 0) {
        double b = bv[0];
        int p = bi[0];
        for (int q = 1; q < 4; ++q)
          if (gj_better(bv[q], bi[q], b, p)) {
            b = bv[q];
            p = bi[q];
          }
        sh_win = p;
        sh_best = b;
      }
      __syncthreads();
      if (!multi) {
        if (gi == sh_win) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) prow[q] = a[q];
        }
        if (gi == gc) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) rowgc[q] = a[q];
        }
        if (tid == 0) sh_p = sh_win;
        __syncthreads();
      } else {
        zd* slot = t.slots + (int64_t)(gc & 1) * slen;
        if (tid == 0) slot[(int64_t)w * (kGjNb + 1)] = zd{sh_best, (double)sh_win};
        if (gi == sh_win) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) slot[(int64_t)w * (kGjNb + 1) + 1 + q] = a[q];
        }
        if (gi == gc) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) slot[(int64_t)t.wpt * (kGjNb + 1) + q] = a[q];
        }
        __syncthreads();
        if (tid == 0) {
          // release (a write-back, no invalidate): the slot writes above precede the count
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(t.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int target = t.wpt * (gc + 1);
          int64_t spins = 0;
          // relaxed polling (an acquire load would invalidate the caches at every poll); the
          // fence after the loop orders what follows
          while (__hip_atomic_load(t.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kGjSpinLimit) {
              __hip_atomic_store(t.info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // an invalidate, no write-back
          double b = -1.0;
          int p = 0x7fffffff, pw = 0;
          for (int u = 0; u < t.wpt; ++u) {
            const zd c = slot[(int64_t)u * (kGjNb + 1)];
            const int ci = (int)c.im;
            if (gj_better(c.re, ci, b, p)) {
              b = c.re;
              p = ci;
              pw = u;
            }
          }
          sh_p = p;
          sh_best = b;
          sh_win = pw;
        }
        __syncthreads();
        if (tid < kGjNb) {
          prow[tid] = slot[(int64_t)sh_win * (kGjNb + 1) + 1 + tid];
          rowgc[tid] = slot[(int64_t)t.wpt * (kGjNb + 1) + tid];
        }
        __syncthreads();
      }
      int p = sh_p;
      if (p >= n) p = gc;
      if (w == 0 && tid == 0) {
        t.piv[gc] = p;
        if (!(sh_best > 0.0) && *t.info == 0) *t.info = gc + 1;
      }
      // the pivot row moves to position gc, the row from gc to position p
      if (p != gc) {
        if (gi == gc) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) a[q] = prow[q];
        } else if (gi == p) {
  #pragma unroll
          for (int q = 0; q < kGjNb; ++q) a[q] = rowgc[q];
        }
      }
      const zd pv = prow[j];
      const zd inv = (zabs2(pv) > 0.0) ? zdiv(zd{1.0, 0.0}, pv) : zd{0.0, 0.0};
      if (gi == gc) {
  #pragma unroll
        for (int q = 0; q < kGjNb; ++q) a[q] = (q == j) ? inv : zmul(prow[q], inv);
      } else if (own) {
        zd f = a[0];
#pragma unroll
        for (int q = 1; q < kGjNb; ++q)
          if (q == j) f = a[q];
  #pragma unroll
        for (int q = 0; q < kGjNb; ++q) {
          if (q == j)
            a[q] = zd{-(f.re * inv.re - f.im * inv.im), -(f.re * inv.im + f.im * inv.re)};
          else
            a[q] = zsub(a[q], zmul(f, zmul(prow[q], inv)));
        }
      }
      __syncthreads();
    }
  }
  if (own) {
#pragma unroll
    for (int q = 0; q < kGjNb; ++q)
      if (q < nb) A[gi + (int64_t)(j0 + q) * lda] = a[q];
  }
}

// Gauss-Jordan inversion of a batch of matrices of up to NT rows, several workgroups per
// matrix, one launch for the whole inversion. Pivoting is implicit: rows are never moved;
// the pivot of column j is the unused row pi(j) of largest modulus (ties to the smaller
// row), and the in-place result M satisfies inv(A)[j, c] = M[pi(j), pi^-1(c)]. Every
// workgroup of a matrix factors each panel of kGjNb columns itself (one row per thread,
// in registers; identical arithmetic, so identical results), then applies the panel to the
// columns it owns (panels assigned round-robin):
//   A[:, c] += T W[:, c] - E W[:, c],  W = A[pi(J), c] staged in LDS,
// with T the transformed panel and E the rows pi(J). Finally each workgroup gathers its
// share of the inverse into out.
//
// Workgroups of a matrix synchronise per panel through sync words (zeroed by the host;
// 2 npan + 1 per matrix), not through full barriers:
//   ready[p]  the owner of panel p has applied every earlier panel to p's columns. The
//             owner updates the next panel's columns first (look-ahead) and raises the
//             flag at once, so the rest of its update overlaps the next panel's pivoting;
//   reads[p]  workgroups other than the owner that have loaded panel p: the owner stores
//             the transformed panel only once all of them have it in registers;
//   done      arrivals before the final gather, which reads every workgroup's columns.
// Waits are bounded (cooperative launch: all workgroups are resident); on time-out
// info = -1.
constexpr int kGjChunk = 16;
constexpr int64_t kGjCoopSpin = int64_t(1) << 22;

// thread 0 waits until *w >= target, then the workgroup continues (acquire). The flag is
// polled with relaxed loads (an acquire load would invalidate the caches at every poll, also
// for the other workgroups on the same XCD); the fence after the loop orders what follows.
__device__ inline void gj_wait_at_least(int32_t* w, int target, int32_t* info) {
  if (threadIdx.x == 0) {
    int64_t spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kGjCoopSpin) {
        __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // acquire: the signaller's writes before its release are visible to this workgroup's
    // reads after the barrier below (an invalidate, no write-back)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// after a workgroup barrier: thread 0 publishes the workgroup's prior memory operations
// (callers pass a workgroup barrier first, so that every thread's writes precede the release)
__device__ inline void gj_signal(int32_t* w) {
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // a write-back, no invalidate
    __hip_atomic_fetch_add(w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// complex helpers as fused multiply-adds (four per complex product)
__device__ inline void gj_fma(zd& acc, const zd& a, const zd& b) {  // acc += a b
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
__device__ inline zd gj_fms(const zd& a, const zd& f, const zd& c) {  // a - f c
  return zd{fma(-f.re, c.re, fma(f.im, c.im, a.re)), fma(-f.re, c.im, fma(-f.im, c.re, a.im))};
}
__device__ inline zd gj_mul(const zd& a, const zd& b) {
  return zd{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

// NT threads per workgroup, RPT rows per thread (rows tid + r NT), panels of NB columns
template <int RPT, int NB, int NT>
__global__ void __launch_bounds__(NT) gj_coop_kernel(const GjCoopTask* __restrict__ tasks, int ntasks) {
  constexpr int NW = NT / 64, NR = NT * RPT;
  const int64_t u = blockIdx.x;
  const GjCoopTask t = tasks[find_task(tasks, ntasks, u)];
  const int w = (int)(u - t.unit_begin);
  const int nwg = t.nwg;
  const int n = t.n;
  const int64_t lda = t.lda;
  zd* A = t.A;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // per column: each wave's best candidate (value, row, the row itself); two slots
  // alternate between even and odd columns
  __shared__ double cv[2][NW];
  __shared__ int ci[2][NW];
  __shared__ zd crow[2][NW][NB];
  __shared__ int pivl[NR], idx[NR];
  __shared__ zd Ws[NB][NB + 1];
  const int npan = (n + NB - 1) / NB;
  int32_t* ready = t.counter;
  int32_t* reads = t.counter + npan;
  int32_t* done = t.counter + 2 * npan;
  bool used[RPT];  // the row has been a pivot
#pragma unroll
  for (int r = 0; r < RPT; ++r) used[r] = false;

  // apply panel (j0, nb) to the columns of panel pc; myq[r]: row r is pi(j0 + myq[r]), or -1
  auto update_panel = [&](int pc, int j0, int nb, const zd (&a)[RPT][NB], const int (&myq)[RPT]) {
    const int c0 = pc * NB;
    for (int e = tid; e < NB * NB; e += NT) {
      const int q = e % NB, cc = e / NB, c = c0 + cc;
      Ws[q][cc] = (q < nb && c < n) ? A[pivl[j0 + q] + (int64_t)c * lda] : zd{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int row = tid + r * NT;
      if (row < n) {
        zd acc[NB];
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
          const int c = c0 + cc;
          acc[cc] = (c < n) ? A[row + (int64_t)c * lda] : zd{0.0, 0.0};
        }
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
#pragma unroll
          for (int q = 0; q < NB; ++q) gj_fma(acc[cc], a[r][q], Ws[q][cc]);
          if (myq[r] >= 0) acc[cc] = zsub(acc[cc], Ws[myq[r]][cc]);
        }
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
          const int c = c0 + cc;
          if (c < n) A[row + (int64_t)c * lda] = acc[cc];
        }
      }
    }
    __syncthreads();
  };

  for (int pn = 0; pn < npan; ++pn) {
    const int j0 = pn * NB, nb = min(NB, n - j0);
    const int owner = pn % nwg;
    // panel pn must be final; its owner made it so itself
    if (nwg > 1 && pn > 0 && owner != w) gj_wait_at_least(ready + pn, 1, t.info);
    zd a[RPT][NB];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int row = tid + r * NT;
#pragma unroll
      for (int q = 0; q < NB; ++q)
        a[r][q] = (row < n && q < nb) ? A[row + (int64_t)(j0 + q) * lda] : zd{0.0, 0.0};
    }
    if (nwg > 1 && owner != w) {
      __syncthreads();  // every thread's loads of the panel have completed
      gj_signal(reads + pn);
    }
    int myq[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) myq[r] = -1;
    // one workgroup barrier per column; the column loop is unrolled so that the register
    // rows are indexed by constants only
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < nb) {
        const int gc = j0 + j, par = j & 1;
        double best = -1.0;
        int besti = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int row = tid + r * NT;
          if (row < n && !used[r]) {
            const double v = zabs2(a[r][j]);
            if (gj_better(v, row, best, besti)) {
              best = v;
              besti = row;
            }
          }
        }
        gj_wave_argmax(best, besti);
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (besti == tid + r * NT) {
#pragma unroll
            for (int q = 0; q < NB; ++q) crow[par][wave][q] = a[r][q];
          }
        if (lane == 0) {
          cv[par][wave] = best;
          ci[par][wave] = besti;
        }
        __syncthreads();
        double b = cv[par][0];
        int p = ci[par][0], pw = 0;
#pragma unroll
        for (int q = 1; q < NW; ++q)
          if (gj_better(cv[par][q], ci[par][q], b, p)) {
            b = cv[par][q];
            p = ci[par][q];
            pw = q;
          }
        // n - gc > 0 rows remain unused, so some wave has a candidate and p < n
        if (tid == 0) pivl[gc] = p;
        if (w == 0 && tid == 0) {
          t.piv[gc] = p;
          if (!(b > 0.0) && *t.info == 0) *t.info = gc + 1;
        }
        zd pr[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) pr[q] = crow[par][pw][q];
        const double d2 = zabs2(pr[j]);
        const double s = d2 > 0.0 ? 1.0 / d2 : 0.0;
        const zd inv{pr[j].re * s, -pr[j].im * s};
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int row = tid + r * NT;
          if (row == p) {
            used[r] = true;
            myq[r] = j;
#pragma unroll
            for (int q = 0; q < NB; ++q) a[r][q] = (q == j) ? inv : gj_mul(a[r][q], inv);
          } else if (row < n) {
            const zd fi = gj_mul(a[r][j], inv);
#pragma unroll
            for (int q = 0; q < NB; ++q) a[r][q] = (q == j) ? zd{-fi.re, -fi.im} : gj_fms(a[r][q], fi, pr[q]);
          }
        }
      }
    }
    __syncthreads();
    // the owner stores the transformed panel once every other workgroup has loaded it
    if (owner == w) {
      if (nwg > 1) gj_wait_at_least(reads + pn, nwg - 1, t.info);
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int row = tid + r * NT;
        if (row < n) {
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < nb) A[row + (int64_t)(j0 + q) * lda] = a[r][q];
        }
      }
      __syncthreads();
    }
    // look-ahead: the next panel's columns first, then its flag, then the other columns
    const int la = pn + 1;
    if (la < npan && la % nwg == w) {
      update_panel(la, j0, nb, a, myq);
      if (nwg > 1) gj_signal(ready + la);
    }
    for (int pc = w; pc < npan; pc += nwg)
      if (pc != pn && pc != la) update_panel(pc, j0, nb, a, myq);
  }
  // every workgroup's columns are final before any reads them below
  if (nwg > 1) {
    __syncthreads();
    gj_signal(done);
    gj_wait_at_least(done, nwg, t.info);
  }
  // inv(A)[j, c] = M[pi(j), pi^-1(c)]: this workgroup's columns of out
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int row = tid + r * NT;
    if (row < n) idx[pivl[row]] = row;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int row = tid + r * NT;
    if (row < n)
      for (int pc = w; pc < npan; pc += nwg)
        for (int c = pc * NB; c < min(n, pc * NB + NB); ++c)
          t.out[row + (int64_t)c * n] = A[pivl[row] + (int64_t)idx[c] * lda];
  }
}

// ---- stepped Gauss-Jordan: one launch per panel (see GjStepArgs)
constexpr int kStepRpt = kGjStepMax / kGjStepThreads;  // rows per thread of workgroup 0
constexpr int kStepCols = 8;                           // columns per updating workgroup

__global__ void __launch_bounds__(kGjStepThreads) gj_step_kernel(GjStepArgs g, int j) {
  constexpr int NB = kGjStepNb, NT = kGjStepThreads, NW = NT / 64, RPT = kStepRpt;
  const int n = g.n;
  const int64_t lda = g.lda;
  zd* A = g.A;
  const int npan = (n + NB - 1) / NB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j0 = j * NB, nb = j >= 0 ? min(NB, n - j0) : 0;  // panel j, applied in this step
  __shared__ zd W[NB][kStepCols + 1];                        // panel j's pivot rows, block's columns
  if (blockIdx.x == 0) {
    // ---- panel j + 1: apply panel j to its columns, then factor it
    const int jn = j + 1;
    if (jn >= npan) return;
    const int k0 = jn * NB, kb = min(NB, n - k0);
    __shared__ double cv[2][NW];
    __shared__ int ci[2][NW];
    __shared__ zd crow[2][NW][NB];
    zd a[RPT][NB];
    bool used[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int row = tid + r * NT;
      used[r] = row >= n || g.rowcol[row] >= 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) a[r][q] = (row < n && q < kb) ? A[row + (int64_t)(k0 + q) * lda] : zd{0.0, 0.0};
    }
    if (nb > 0) {
      for (int e = tid; e < NB * NB; e += NT) {
        const int pp = e / NB, q = e % NB;
        W[pp][q] = (pp < nb && q < kb) ? A[g.piv[j0 + pp] + (int64_t)(k0 + q) * lda] : zd{0.0, 0.0};
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int row = tid + r * NT;
        if (row >= n) continue;
        zd tr[NB];
#pragma unroll
        for (int pp = 0; pp < NB; ++pp) tr[pp] = pp < nb ? A[row + (int64_t)(j0 + pp) * lda] : zd{0.0, 0.0};
        const int rc = g.rowcol[row];
        const int qi = (rc >= j0 && rc < j0 + nb) ? rc - j0 : -1;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
#pragma unroll
          for (int pp = 0; pp < NB; ++pp) gj_fma(a[r][q], tr[pp], W[pp][q]);
          if (qi >= 0) a[r][q] = zsub(a[r][q], W[qi][q]);
        }
      }
    }
    // factor panel j + 1: one workgroup barrier per column (as in gj_coop_kernel)
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
      if (jj < kb) {
        const int gc = k0 + jj, par = jj & 1;
        double best = -1.0;
        int besti = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int row = tid + r * NT;
          if (!used[r]) {
            const double v = zabs2(a[r][jj]);
            if (gj_better(v, row, best, besti)) {
              best = v;
              besti = row;
            }
          }
        }
        gj_wave_argmax(best, besti);
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (besti == tid + r * NT) {
#pragma unroll
            for (int q = 0; q < NB; ++q) crow[par][wave][q] = a[r][q];
          }
        if (lane == 0) {
          cv[par][wave] = best;
          ci[par][wave] = besti;
        }
        __syncthreads();
        double b = cv[par][0];
        int p = ci[par][0], pw = 0;
#pragma unroll
        for (int q = 1; q < NW; ++q)
          if (gj_better(cv[par][q], ci[par][q], b, p)) {
            b = cv[par][q];
            p = ci[par][q];
            pw = q;
          }
        // n - gc > 0 rows remain unused, so p < n
        if (tid == 0) {
          g.piv[gc] = p;
          if (!(b > 0.0) && *g.info == 0) *g.info = gc + 1;
        }
        zd pr[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) pr[q] = crow[par][pw][q];
        const double d2 = zabs2(pr[jj]);
        const double sc = d2 > 0.0 ? 1.0 / d2 : 0.0;
        const zd inv{pr[jj].re * sc, -pr[jj].im * sc};
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int row = tid + r * NT;
          if (row == p) {
            used[r] = true;
            g.rowcol[row] = gc;
#pragma unroll
            for (int q = 0; q < NB; ++q) a[r][q] = (q == jj) ? inv : gj_mul(a[r][q], inv);
          } else if (row < n) {
            const zd fi = gj_mul(a[r][jj], inv);
#pragma unroll
            for (int q = 0; q < NB; ++q) a[r][q] = (q == jj) ? zd{-fi.re, -fi.im} : gj_fms(a[r][q], fi, pr[q]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int row = tid + r * NT;
      if (row < n) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < kb) A[row + (int64_t)(k0 + q) * lda] = a[r][q];
      }
    }
    return;
  }
  // ---- the other workgroups: apply panel j to kStepCols columns (all rows), skipping the
  // columns of panels j (the multipliers) and j + 1 (workgroup 0's)
  if (nb == 0) return;
  const int c0 = (blockIdx.x - 1) * kStepCols;
  const int s0 = (j + 1) * NB, s1 = min(n, s0 + NB);
  for (int e = tid; e < NB * kStepCols; e += NT) {
    const int pp = e / kStepCols, cc = e % kStepCols, c = c0 + cc;
    W[pp][cc] = (pp < nb && c < n) ? A[g.piv[j0 + pp] + (int64_t)c * lda] : zd{0.0, 0.0};
  }
  __syncthreads();  // every pivot-row value is read before any row of these columns changes
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int row = tid + r * NT;
    if (row >= n) continue;
    zd tr[NB];
#pragma unroll
    for (int pp = 0; pp < NB; ++pp) tr[pp] = pp < nb ? A[row + (int64_t)(j0 + pp) * lda] : zd{0.0, 0.0};
    const int rc = g.rowcol[row];
    const int qi = (rc >= j0 && rc < j0 + nb) ? rc - j0 : -1;
    for (int cc = 0; cc < kStepCols; ++cc) {
      const int c = c0 + cc;
      if (c >= n) break;
      if ((c >= j0 && c < j0 + nb) || (c >= s0 && c < s1)) continue;
      zd v = A[row + (int64_t)c * lda];
#pragma unroll
      for (int pp = 0; pp < NB; ++pp) gj_fma(v, tr[pp], W[pp][cc]);
      if (qi >= 0) v = zsub(v, W[qi][cc]);
      A[row + (int64_t)c * lda] = v;
    }
  }
}

// out[i, c] = M[piv[i], rowcol[c]]  (grid: row blocks of 256 x columns)
__global__ void __launch_bounds__(256) gj_step_gather_kernel(GjStepArgs g, zd* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (i >= g.n) return;
  out[i + (int64_t)c * g.n] = g.A[g.piv[i] + (int64_t)g.rowcol[c] * g.lda];
}

// Row swaps of the panel applied to columns outside J. grid.x = task, grid.y = column chunk.
__global__ void __launch_bounds__(256) gj_swaps_kernel(const GjTask* __restrict__ tasks, int j0) {
  const GjTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (j0 >= n) return;
  const int nb = min(kGjNb, n - j0);
  const int c = blockIdx.y * 256 + threadIdx.x;
  if (c >= n || (c >= j0 && c < j0 + nb)) return;
  zd* col = t.A + (int64_t)c * t.lda;
  for (int q = 0; q < nb; ++q) {
    const int gc = j0 + q, p = t.piv[gc];
    if (p != gc) {
      zd a = col[gc];
      col[gc] = col[p];
      col[p] = a;
    }
  }
}

__global__ void __launch_bounds__(256) gj_copyrow_kernel(const GjTask* __restrict__ tasks, int j0,
                                                         zd* const* __restrict__ W) {
  const GjTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (j0 >= n) return;
  const int nb = min(kGjNb, n - j0);
  const int c = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int q = threadIdx.x & 15;
  if (c >= n || q >= nb) return;
  W[blockIdx.x][q + (int64_t)c * nb] = t.A[(j0 + q) + (int64_t)c * t.lda];
}

// Row exchanges of the panel on the columns outside J, then the pivot rows into W (all
// columns): one thread per column. grid.x = task, grid.y = column chunk.
__global__ void __launch_bounds__(256) gj_swapcopy_kernel(const GjTask* __restrict__ tasks, int j0,
                                                          zd* const* __restrict__ W) {
  const GjTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (j0 >= n) return;
  const int nb = min(kGjNb, n - j0);
  const int c = blockIdx.y * 256 + threadIdx.x;
  if (c >= n) return;
  zd* col = t.A + (int64_t)c * t.lda;
  if (c < j0 || c >= j0 + nb) {
    for (int q = 0; q < nb; ++q) {
      const int gc = j0 + q, p = t.piv[gc];
      if (p != gc) {
        const zd a = col[gc];
        col[gc] = col[p];
        col[p] = a;
      }
    }
  }
  zd* w = W[blockIdx.x] + (int64_t)c * nb;
  for (int q = 0; q < nb; ++q) w[q] = col[j0 + q];
}

__global__ void __launch_bounds__(256) gj_fixrow_kernel(const GjTask* __restrict__ tasks, int j0,
                                                        zd* const* __restrict__ W) {
  const GjTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (j0 >= n) return;
  const int nb = min(kGjNb, n - j0);
  const int c = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int q = threadIdx.x & 15;
  if (c >= n || q >= nb || (c >= j0 && c < j0 + nb)) return;
  zd* a = t.A + (j0 + q) + (int64_t)c * t.lda;
  *a = zsub(*a, W[blockIdx.x][q + (int64_t)c * nb]);
}

// Compose the column permutation (one thread per task) then gather columns into out.
__global__ void gj_compose_kernel(const GjTask* __restrict__ tasks, int32_t* const* __restrict__ work) {
  const GjTask t = tasks[blockIdx.x];
  if (threadIdx.x != 0) return;
  int32_t* idx = work[blockIdx.x];
  for (int j = 0; j < t.n; ++j) idx[j] = j;
  for (int gc = t.n - 1; gc >= 0; --gc) {
    const int p = t.piv[gc];
    const int a = idx[gc];
    idx[gc] = idx[p];
    idx[p] = a;
  }
}
__global__ void __launch_bounds__(256) gj_gather_kernel(const GjTask* __restrict__ tasks,
                                                        zd* const* __restrict__ out,
                                                        int32_t* const* __restrict__ work) {
  const GjTask t = tasks[blockIdx.x];
  const int j = blockIdx.y;
  if (j >= t.n) return;
  const int src = work[blockIdx.x][j];
  const zd* a = t.A + (int64_t)src * t.lda;
  zd* o = out[blockIdx.x] + (int64_t)j * t.n;
  for (int i = threadIdx.x; i < t.n; i += 256) o[i] = a[i];
}

// ---------------------------------------------------------------------------------------
__device__ inline int seg_of(const NSeg* __restrict__ segs, int64_t base, int nseg, int pos) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[base + mid].off <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <class PT>
__global__ void __launch_bounds__(256) cross_kernel(const CrossTask* __restrict__ tasks, int ntasks,
                                                    const NSeg* __restrict__ segs,
                                                    const PT* __restrict__ pool) {
  const int64_t u = blockIdx.x;
  const int ti = find_task(tasks, ntasks, u);
  const CrossTask t = tasks[ti];
  int64_t lu = u - t.unit_begin;
  const int m = t.m, mn = t.m + t.nN, s = t.s, r = t.m - t.s;
  const int ucol_r = (mn + 63) >> 6, ucol_c = (m + 63) >> 6;
  const int64_t ncol_units = (int64_t)ucol_r * ucol_c;
  const PT* bb = pool + t.tile_bb;
  if (lu < ncol_units) {
    // Ccol: rows (R, S, N), cols (S, R) = perm order
    const int bi = (int)(lu % ucol_r), bj = (int)(lu / ucol_r);
    const int i = bi * 64 + (threadIdx.x & 63);
    if (i >= mn) return;
    int pi = 0;
    const NSeg* sg = nullptr;
    int li = 0;
    if (i < m) {
      pi = (i < r) ? t.perm[s + i] : t.perm[i - r];
    } else {
      sg = segs + t.seg_off + seg_of(segs, t.seg_off, t.nseg, i - m);
      li = sg->live[i - m - sg->off];
    }
    for (int jj = 0; jj < 16; ++jj) {
      const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
      if (j >= m) break;
      const int pj = t.perm[j];
      const zd v = widen((i < m) ? bb[pi + (int64_t)pj * m] : pool[sg->tile_nb + li + (int64_t)pj * sg->ld]);
      t.Ccol[i + (int64_t)j * mn] = v;
    }
  } else {
    lu -= ncol_units;
    // Crow: rows (S, R) = perm order, cols (R, S, N)
    const int urow_r = (m + 63) >> 6;
    const int bi = (int)(lu % urow_r), bj = (int)(lu / urow_r);
    const int i = bi * 64 + (threadIdx.x & 63);
    if (i >= m) return;
    const int pi = t.perm[i];
    for (int jj = 0; jj < 16; ++jj) {
      const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
      if (j >= mn) break;
      zd v;
      if (j < m) {
        const int pj = (j < r) ? t.perm[s + j] : t.perm[j - r];
        v = widen(bb[pi + (int64_t)pj * m]);
      } else {
        const NSeg& sg = segs[t.seg_off + seg_of(segs, t.seg_off, t.nseg, j - m)];
        v = widen(pool[sg.tile_bn + pi + (int64_t)sg.live[j - m - sg.off] * m]);
      }
      t.Crow[i + (int64_t)j * m] = v;
    }
  }
}

__global__ void __launch_bounds__(256) extract_r_kernel(const ExtractTask* __restrict__ tasks) {
  const ExtractTask t = tasks[blockIdx.x];
  const int j = blockIdx.y;
  if (j >= t.m) return;
  for (int i = threadIdx.x; i < t.m; i += 256) {
    zd v{0.0, 0.0};
    if (i <= j && i < t.rows) v = t.M[i + (int64_t)j * t.rows];
    t.R[i + (int64_t)j * t.m] = v;
  }
}

// copies and transposes in one launch (t.transpose, uniform per task); units of 64 x 64
template <class DT>
__global__ void __launch_bounds__(256) copy_kernel(const CopyTask* __restrict__ tasks, int ntasks) {
  __shared__ zd tile[64][65];
  const int64_t u = blockIdx.x;
  const int ti = find_task(tasks, ntasks, u);
  const CopyTask t = tasks[ti];
  const int64_t lu = u - t.unit_begin;
  const int nbr = (t.rows + 63) >> 6;
  const int bi = (int)(lu % nbr), bj = (int)(lu / nbr);
  if (t.transpose) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int q = ty; q < 64; q += 4) {
      const int i = bi * 64 + tx, j = bj * 64 + q;
      if (i < t.rows && j < t.cols) tile[q][tx] = t.src[i + (int64_t)j * t.lds];
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
      const int j = bj * 64 + tx, i = bi * 64 + q;
      if (i < t.rows && j < t.cols) static_cast<DT*>(t.dst)[j + (int64_t)i * t.ldd] = narrow<DT>(tile[tx][q]);
    }
    return;
  }
  const int i = bi * 64 + (threadIdx.x & 63);
  if (i >= t.rows) return;
  for (int jj = 0; jj < 16; ++jj) {
    const int j = bj * 64 + (threadIdx.x >> 6) + 4 * jj;
    if (j >= t.cols) break;
    static_cast<DT*>(t.dst)[i + (int64_t)j * t.ldd] = narrow<DT>(t.src[i + (int64_t)j * t.lds]);
  }
}

}  // namespace


void launch_sum_parts(const SumTask* tasks, int ntasks, int64_t nunits, hipStream_t st) {
  if (ntasks <= 0 || nunits <= 0) return;
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)nunits), dim3(256), 0, st, tasks, ntasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_pchol(const PcholTask* tasks, int ntasks, int mmax, double eps, hipStream_t st) {
  if (ntasks <= 0) return;
  // dynamic LDS: [mult (16 B)] + dg (8 B) + pos, pv (4 B each) per column; 64 KB in all
  // with the static part (about 17 KB)
  constexpr size_t kBudget = 65536 - 17664;
  const size_t with_mult = (size_t)mmax * 32, without = (size_t)mmax * 16;
  if (without > kBudget) throw Error(FMMLU_EINVAL, "ID block wider than " + std::to_string(kBudget / 16));
  const int in_lds = with_mult <= kBudget ? 1 : 0;
  // 256 threads up to 128 columns (two or more row slices per column), 1024 beyond
  if (mmax <= 128)
    hipLaunchKernelGGL(pchol_kernel<256>, dim3(ntasks), dim3(256), in_lds ? with_mult : without, st, tasks, eps,
                       in_lds);
  else
    hipLaunchKernelGGL(pchol_kernel<kPcholThreads>, dim3(ntasks), dim3(kPcholThreads), in_lds ? with_mult : without, st,
                       tasks, eps, in_lds);
  FMMLU_HIP(hipGetLastError());
}

void launch_pchol_t(const PcholTask* tasks, int ntasks, int mmax, hipStream_t st) {
  if (ntasks <= 0) return;
  // back substitution: NC right-hand-side columns per workgroup, s x NC in LDS
  const dim3 grid_of_nc[4] = {dim3(ntasks, (mmax + 7) / 8), dim3(ntasks, (mmax + 3) / 4),
                              dim3(ntasks, (mmax + 1) / 2), dim3(ntasks, mmax)};
  if (mmax <= 480)
    hipLaunchKernelGGL(pchol_t_kernel<8>, grid_of_nc[0], dim3(256), (size_t)mmax * 8 * sizeof(zd), st, tasks);
  else if (mmax <= 960)
    hipLaunchKernelGGL(pchol_t_kernel<4>, grid_of_nc[1], dim3(256), (size_t)mmax * 4 * sizeof(zd), st, tasks);
  else if (mmax <= 1920)
    hipLaunchKernelGGL(pchol_t_kernel<2>, grid_of_nc[2], dim3(256), (size_t)mmax * 2 * sizeof(zd), st, tasks);
  else
    hipLaunchKernelGGL(pchol_t_kernel<1>, grid_of_nc[3], dim3(256), (size_t)mmax * sizeof(zd), st, tasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_pchol_block(const PcholTask* tasks, int ntasks, int k0, double eps, hipStream_t st, int mmax) {
  if (ntasks <= 0) return;
  if (mmax > kPcholThreadsB) throw Error(FMMLU_EINVAL, "blocked pivoted Cholesky takes m <= 1024");
  // one column per thread: the fewest wavefronts that cover the widest matrix (cheaper
  // barriers and pivot searches per step)
  if (mmax <= 256)
    hipLaunchKernelGGL(pchol_block_kernel<256>, dim3(ntasks), dim3(256), 0, st, tasks, k0, eps);
  else if (mmax <= 512)
    hipLaunchKernelGGL(pchol_block_kernel<512>, dim3(ntasks), dim3(512), 0, st, tasks, k0, eps);
  else
    hipLaunchKernelGGL(pchol_block_kernel<1024>, dim3(ntasks), dim3(1024), 0, st, tasks, k0, eps);
  FMMLU_HIP(hipGetLastError());
}

void launch_pchol_finish(const PcholTask* tasks, int ntasks, int mmax, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(pchol_finish_kernel, dim3(ntasks, (unsigned)std::max(1, (mmax + 31) / 32)), dim3(kPcholThreads),
                     (size_t)mmax * sizeof(int), st, tasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_reduce_tw(const RedTwTask* tasks, int ntasks, int nmax, hipStream_t st) {
  if (ntasks <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(reduce_tw_kernel, dim3(ntasks, (nmax + 255) / 256), dim3(256), 0, st, tasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_qr_panel(const QrTask* tasks, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(qr_panel_kernel, dim3(ntasks), dim3(256), 0, st, tasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_cpqr(const CpqrTask* tasks, int ntasks, int mmax, double eps, hipStream_t st) {
  if (ntasks <= 0) return;
  if ((size_t)mmax * sizeof(double) > 65536) throw Error(FMMLU_EINVAL, "CPQR block wider than 8192");
  hipLaunchKernelGGL(cpqr_kernel, dim3(ntasks), dim3(256), (size_t)mmax * sizeof(double), st, tasks, eps);
  FMMLU_HIP(hipGetLastError());
}

// While several factorizations run at once (on several host threads and streams), at most one
// cooperative kernel may be in flight: two partially resident cooperative grids could each
// wait for the other's compute units. The launch then holds a process-wide lock until the
// kernel has finished.
namespace {
std::atomic<int> g_active_factorizations{0};
std::mutex g_coop_mutex;

template <class F>
void coop_launch(F&& launch, hipStream_t st) {
  if (g_active_factorizations.load() > 1) {
    std::lock_guard<std::mutex> lk(g_coop_mutex);
    launch();
    FMMLU_HIP(hipStreamSynchronize(st));
  } else {
    launch();
  }
}
}  // namespace

ActiveFactorization::ActiveFactorization() { ++g_active_factorizations; }
ActiveFactorization::~ActiveFactorization() { --g_active_factorizations; }
int ActiveFactorization::count() { return g_active_factorizations.load(); }

void launch_gj_panel(const GjTask* tasks, int ntasks, int j0, int wmax, hipStream_t st) {
  if (ntasks <= 0) return;
  if (wmax <= 1) {
    hipLaunchKernelGGL(gj_panel_kernel, dim3(ntasks, 1), dim3(kGjPanelRows), 0, st, tasks, j0);
  } else {
    void* args[] = {(void*)&tasks, (void*)&j0};
    coop_launch(
        [&]() {
          FMMLU_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(gj_panel_kernel), dim3(ntasks, wmax),
                                               dim3(kGjPanelRows), args, 0, st));
        },
        st);
  }
  FMMLU_HIP(hipGetLastError());
}

// (rows per thread, panel width, threads) for matrices of up to nmax rows: one row per
// thread, 256 threads up to 256 rows, 512 beyond
template <class F>
void gj_coop_dispatch(int nmax, F&& f) {
  if (nmax <= 256)
    f(reinterpret_cast<const void*>(gj_coop_kernel<1, 16, 256>), 256);
  else
    f(reinterpret_cast<const void*>(gj_coop_kernel<1, 16, 512>), 512);
}

void launch_gj_coop(const GjCoopTask* tasks, int ntasks, int64_t nwg_total, int nmax, hipStream_t st) {
  if (ntasks <= 0 || nwg_total <= 0) return;
  if (nmax > kGjCoopMax) throw Error(FMMLU_EINVAL, "cooperative Gauss-Jordan takes n <= 512");
  void* args[] = {(void*)&tasks, (void*)&ntasks};
  // one workgroup per matrix: nothing waits across workgroups, an ordinary launch suffices
  const bool independent = nwg_total == ntasks;
  gj_coop_dispatch(nmax, [&](const void* k, int nt) {
    if (independent)
      FMMLU_HIP(hipLaunchKernel(k, dim3((unsigned)nwg_total), dim3(nt), args, 0, st));
    else
      coop_launch([&]() { FMMLU_HIP(hipLaunchCooperativeKernel(k, dim3((unsigned)nwg_total), dim3(nt), args, 0, st)); },
                  st);
  });
  FMMLU_HIP(hipGetLastError());
}

int gj_coop_capacity(int nmax) {
  int dev = 0, per_cu = 0, cus = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  FMMLU_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  gj_coop_dispatch(nmax, [&](const void* k, int nt) {
    FMMLU_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, nt, 0));
  });
  return per_cu * cus;
}

void launch_gj_step(const GjStepArgs& a, int j, hipStream_t st) {
  if (a.n <= 0) return;
  if (a.n > kGjStepMax) throw Error(FMMLU_EINVAL, "stepped Gauss-Jordan takes n <= 2048");
  const int ncb = (a.n + kStepCols - 1) / kStepCols;
  hipLaunchKernelGGL(gj_step_kernel, dim3(1 + ncb), dim3(kGjStepThreads), 0, st, a, j);
  FMMLU_HIP(hipGetLastError());
}

void launch_gj_step_gather(const GjStepArgs& a, zd* out, hipStream_t st) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(gj_step_gather_kernel, dim3((a.n + 255) / 256, a.n), dim3(256), 0, st, a, out);
  FMMLU_HIP(hipGetLastError());
}

int gj_panel_capacity() {
  int dev = 0, per_cu = 0, cus = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  FMMLU_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  FMMLU_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(gj_panel_kernel),
                                                         kGjPanelRows, 0));
  return per_cu * cus;
}

int gj_coop_cus() {
  int dev = 0, cus = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  FMMLU_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus;
}

void launch_gj_swaps(const GjTask* tasks, int ntasks, int j0, int nmax, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(gj_swaps_kernel, dim3(ntasks, (nmax + 255) / 256), dim3(256), 0, st, tasks, j0);
  FMMLU_HIP(hipGetLastError());
}

void launch_gj_copyrow(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W,
                       hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(gj_copyrow_kernel, dim3(ntasks, (nmax + 15) / 16), dim3(256), 0, st, tasks, j0, W);
  FMMLU_HIP(hipGetLastError());
}

void launch_gj_swapcopy(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(gj_swapcopy_kernel, dim3(ntasks, (nmax + 255) / 256), dim3(256), 0, st, tasks, j0, W);
  FMMLU_HIP(hipGetLastError());
}

void launch_gj_fixrow(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W,
                      hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(gj_fixrow_kernel, dim3(ntasks, (nmax + 15) / 16), dim3(256), 0, st, tasks, j0, W);
  FMMLU_HIP(hipGetLastError());
}

void launch_gj_unpermute(const GjTask* tasks, int ntasks, int nmax, zd* const* out,
                         int32_t* const* work, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(gj_compose_kernel, dim3(ntasks), dim3(64), 0, st, tasks, work);
  FMMLU_HIP(hipGetLastError());
  hipLaunchKernelGGL(gj_gather_kernel, dim3(ntasks, nmax), dim3(256), 0, st, tasks, out, work);
  FMMLU_HIP(hipGetLastError());
}

void launch_gather_cross(const CrossTask* tasks, int ntasks, int64_t nunits, const NSeg* segs,
                         const void* pool, bool pool32, hipStream_t st) {
  if (ntasks <= 0 || nunits <= 0) return;
  if (pool32)
    hipLaunchKernelGGL(cross_kernel<zf>, dim3((unsigned)nunits), dim3(256), 0, st, tasks, ntasks, segs,
                       static_cast<const zf*>(pool));
  else
    hipLaunchKernelGGL(cross_kernel<zd>, dim3((unsigned)nunits), dim3(256), 0, st, tasks, ntasks, segs,
                       static_cast<const zd*>(pool));
  FMMLU_HIP(hipGetLastError());
}

void launch_extract_r(const ExtractTask* tasks, int ntasks, int mmax, hipStream_t st) {
  if (ntasks <= 0 || mmax <= 0) return;
  hipLaunchKernelGGL(extract_r_kernel, dim3(ntasks, mmax), dim3(256), 0, st, tasks);
  FMMLU_HIP(hipGetLastError());
}

void launch_copy(const CopyTask* tasks, int ntasks, int64_t nunits, bool dst32, hipStream_t st) {
  if (ntasks <= 0 || nunits <= 0) return;
  if (dst32)
    hipLaunchKernelGGL(copy_kernel<zf>, dim3((unsigned)nunits), dim3(256), 0, st, tasks, ntasks);
  else
    hipLaunchKernelGGL(copy_kernel<zd>, dim3((unsigned)nunits), dim3(256), 0, st, tasks, ntasks);
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
