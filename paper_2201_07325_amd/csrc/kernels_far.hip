// Far-field pattern operator of the combined-field potential. Section 6.3 defines the
// pattern by u(x) = e^{ikr}/r F(x^) + O(1/r^2); the large-|x| form of the kernel
// (grad_y G -> -ik x^ G, G -> e^{ik|x|}/(4 pi |x|) e^{-ik x^.y}) gives, for
// u = sum_j K(x, x_j) sqrt(w_j) sigma~_j,
//   C[m, j] = (-i / 4 pi) sqrt(w_j) (k d_m.n_j + eta) e^{-ik d_m.x_j},
//   dC/dk   = (-i / 4 pi) sqrt(w_j) (d_m.n_j - i (d_m.x_j)(k d_m.n_j + eta)) e^{-ik d_m.x_j},
//   dC/deta = (-i / 4 pi) sqrt(w_j) e^{-ik d_m.x_j}.
// Geometry is read in tree order; vectors are in the caller's point order and reached
// through the tree-order permutation. Products with C have few rows (directions) and many
// columns, so a workgroup sums one direction over a slice of points and a second pass adds
// the slices in a fixed order; products with C^H give each thread one point.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

// entry of C (op 0), dC/dk (op 2) or dC/deta (op 3) for direction (dx, dy, dz) and tree point j
__device__ inline zd far_entry(const double* __restrict__ p, int64_t n, double k, double eta, int op,
                               double ux, double uy, double uz, int64_t j) {
  const double t = ux * p[j] + uy * p[n + j] + uz * p[2 * n + j];
  const double dn = ux * p[3 * n + j] + uy * p[4 * n + j] + uz * p[5 * n + j];
  const double sw = p[6 * n + j];
  double s, c;
  sincos(k * t, &s, &c);
  const zd e{c, -s};  // e^{-ik t}
  zd a;
  if (op == 0) {
    a = zd{k * dn + eta, 0.0};
  } else if (op == 2) {
    a = zd{dn, -t * (k * dn + eta)};
  } else {
    a = zd{1.0, 0.0};
  }
  return zmul(zd{0.0, -kInv4Pi * sw}, zmul(a, e));
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// part[m * nchunk + c] = sum over tree points j of slice c of entry(m, j) * v[order[j]]
__global__ void __launch_bounds__(256) farfield_fwd_kernel(DevGeom g, int op, const double* __restrict__ dirs,
                                                           int64_t ndir, const int64_t* __restrict__ order,
                                                           const zd* __restrict__ v, zd* __restrict__ part,
                                                           int64_t chunk, int nchunk) {
  __shared__ zd red[4];
  const int64_t m = blockIdx.x;
  const int c = blockIdx.y;
  const double ux = dirs[m], uy = dirs[ndir + m], uz = dirs[2 * ndir + m];
  const int64_t j0 = (int64_t)c * chunk;
  const int64_t j1 = min(g.n, j0 + chunk);
  zd acc{0.0, 0.0};
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const zd e = far_entry(g.p, g.n, g.k, g.eta, op, ux, uy, uz, j);
    zfma(acc, e, v[order[j]]);
  }
  acc.re = wave_sum(acc.re);
  acc.im = wave_sum(acc.im);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[m * nchunk + c] = zadd(zadd(red[0], red[1]), zadd(red[2], red[3]));
}

__global__ void __launch_bounds__(256) farfield_sum_kernel(const zd* __restrict__ part, int64_t ndir, int nchunk,
                                                           zd* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= ndir) return;
  zd s{0.0, 0.0};
  for (int c = 0; c < nchunk; ++c) s = zadd(s, part[m * nchunk + c]);
  out[m] = s;
}

// out[order[j]] = sum_m conj(C[m, j]) v[m]; directions and v staged through LDS
__global__ void __launch_bounds__(256) farfield_adj_kernel(DevGeom g, const double* __restrict__ dirs,
                                                           int64_t ndir, const int64_t* __restrict__ order,
                                                           const zd* __restrict__ v, zd* __restrict__ out) {
  __shared__ double sd[3][256];
  __shared__ zd sv[256];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = j < g.n;
  zd acc{0.0, 0.0};
  for (int64_t m0 = 0; m0 < ndir; m0 += 256) {
    __syncthreads();
    const int64_t ml = m0 + threadIdx.x;
    for (int a = 0; a < 3; ++a) sd[a][threadIdx.x] = ml < ndir ? dirs[a * ndir + ml] : 0.0;
    sv[threadIdx.x] = ml < ndir ? v[ml] : zd{0.0, 0.0};
    __syncthreads();
    if (!live) continue;
    const int cnt = (int)min<int64_t>(256, ndir - m0);
    for (int mm = 0; mm < cnt; ++mm) {
      const zd e = far_entry(g.p, g.n, g.k, g.eta, 0, sd[0][mm], sd[1][mm], sd[2][mm], j);
      zfma(acc, zd{e.re, -e.im}, sv[mm]);
    }
  }
  if (live) out[order[j]] = acc;
}

}  // namespace

int farfield_chunks(int64_t n) { return (int)((n + kFarChunk - 1) / kFarChunk); }

void launch_farfield(const DevGeom& g, int op, const double* dirs, int64_t ndir, const int64_t* order,
                     const zd* in, zd* out, zd* part, hipStream_t st) {
  if (op == 1) {
    if (g.n <= 0) return;
    hipLaunchKernelGGL(farfield_adj_kernel, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, g, dirs, ndir,
                       order, in, out);
    FMMLU_HIP(hipGetLastError());
    return;
  }
  const int nchunk = farfield_chunks(g.n);
  if (ndir <= 0) return;
  hipLaunchKernelGGL(farfield_fwd_kernel, dim3((unsigned)ndir, (unsigned)nchunk), dim3(256), 0, st, g, op, dirs,
                     ndir, order, in, part, (int64_t)kFarChunk, nchunk);
  FMMLU_HIP(hipGetLastError());
  hipLaunchKernelGGL(farfield_sum_kernel, dim3((unsigned)((ndir + 255) / 256)), dim3(256), 0, st, part, ndir,
                     nchunk, out);
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
