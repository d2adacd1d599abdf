// Sweeps of the factored inverse (Section 4.2):
//   A^{-1} ~ (W_1^{-1} ... W_M^{-1}) P_t D^{-1} P_t^T (V_M^{-1} ... V_1^{-1}),
//   V_i^{-1} = L E P^T applied as  x_R -= T^T x_S ;  x_{S u N} -= L_{(S u N)} x_R,
//   W_i^{-1} = P F U   applied as  x_R -= U x_{S u N} ;  x_S -= T x_R,
// with L = X_{(S u N) R} X_RR^{-1} and U = X_RR^{-1} X_{R (S u N)}, and the conjugate
// transposes of the same factors for the adjoint. Boxes of one colour never touch, so a
// colour's boxes run concurrently; their L-updates to shared near DOFs are summed by a
// deterministic gather (scatter_sub) instead of atomics.
//
// These kernels are HBM-bound: every factor byte is read once per sweep.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// x_R of a box is held in dynamic LDS (r complex values, sized by the launch).

// y[i] = sum_k op(A)[i, k] v[k]; N: A is rows x cols (lda), thread per row (coalesced).
__device__ inline zd gemv_n_row(const zd* __restrict__ A, int64_t lda, int i, int cols,
                                const zd* v, bool conjA) {
  zd acc{0.0, 0.0};
  for (int k = 0; k < cols; ++k) {
    zd a = A[i + (int64_t)k * lda];
    if (conjA) a.im = -a.im;
    zfma(acc, a, v[k]);
  }
  return acc;
}

// y[i] = sum_k A[k, i]^(*) v[k] for one i, wavefront-cooperative (lanes over k, coalesced).
__device__ inline zd gemv_t_wave(const zd* __restrict__ A, int64_t lda, int i, int rows,
                                 const zd* v, bool conjA, int lane) {
  zd acc{0.0, 0.0};
  const zd* col = A + (int64_t)i * lda;
  for (int k = lane; k < rows; k += 64) {
    if (conjA)
      zfmac(acc, col[k], v[k]);
    else
      zfma(acc, col[k], v[k]);
  }
  acc.re = wave_sum(acc.re);
  acc.im = wave_sum(acc.im);
  return acc;
}

__global__ void __launch_bounds__(256) solve_fwd_kernel(const SolveBox* __restrict__ boxes, zd* x,
                                                        zd* y, int adjoint) {
  const SolveBox b = boxes[blockIdx.x];
  extern __shared__ zd xr[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // x_R -= T^T x_S  (adjoint: T^H x_S); T is s x r: output i is column i of T
  for (int i = wave; i < b.r; i += 4) {
    zd d{0.0, 0.0};
    const zd* col = b.T + (int64_t)i * b.s;
    for (int l = lane; l < b.s; l += 64) {
      if (adjoint)
        zfmac(d, col[l], x[b.S[l]]);
      else
        zfma(d, col[l], x[b.S[l]]);
    }
    d.re = wave_sum(d.re);
    d.im = wave_sum(d.im);
    if (lane == 0) {
      zd v = zsub(x[b.R[i]], d);
      xr[i] = v;
      x[b.R[i]] = v;
    }
  }
  __syncthreads();
  // y = Lp x_R  (adjoint: Up^H x_R)
  zd* yb = y + b.y_off;
  if (!adjoint) {
    for (int i = threadIdx.x; i < b.nsn; i += 256) yb[i] = gemv_n_row(b.Lp, b.nsn, i, b.r, xr, false);
  } else {
    // Up is r x nsn: output i = sum_k conj(Up[k, i]) xr[k]
    for (int i = wave; i < b.nsn; i += 4) {
      zd d = gemv_t_wave(b.Up, b.r, i, b.r, xr, true, lane);
      if (lane == 0) yb[i] = d;
    }
  }
}

__global__ void __launch_bounds__(256) scatter_sub_kernel(const int32_t* __restrict__ dst,
                                                          const int64_t* __restrict__ ptr,
                                                          const int64_t* __restrict__ src,
                                                          int64_t nd, const zd* __restrict__ y,
                                                          zd* __restrict__ x) {
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= nd) return;
  zd acc{0.0, 0.0};
  for (int64_t q = ptr[d]; q < ptr[d + 1]; ++q) acc = zadd(acc, y[src[q]]);
  const int32_t t = dst[d];
  x[t] = zsub(x[t], acc);
}

__global__ void __launch_bounds__(256) solve_diag_kernel(const SolveBox* __restrict__ boxes, zd* x,
                                                         int adjoint) {
  const SolveBox b = boxes[blockIdx.x];
  extern __shared__ zd xr[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int l = threadIdx.x; l < b.r; l += 256) xr[l] = x[b.R[l]];
  __syncthreads();
  if (!adjoint) {
    for (int i = threadIdx.x; i < b.r; i += 256) x[b.R[i]] = gemv_n_row(b.Xi, b.r, i, b.r, xr, false);
  } else {
    for (int i = wave; i < b.r; i += 4) {
      zd d = gemv_t_wave(b.Xi, b.r, i, b.r, xr, true, lane);
      if (lane == 0) x[b.R[i]] = d;
    }
  }
}

__global__ void __launch_bounds__(256) solve_bwd_kernel(const SolveBox* __restrict__ boxes, zd* x,
                                                        int adjoint) {
  const SolveBox b = boxes[blockIdx.x];
  extern __shared__ zd xr[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // x_R -= U x_SN  (adjoint: Lp^H x_SN)
  if (!adjoint) {
    // Up: r x nsn; thread per output row i, reading x[SN[c]] (gathered on the fly)
    for (int i = threadIdx.x; i < b.r; i += 256) {
      zd acc{0.0, 0.0};
      for (int c = 0; c < b.nsn; ++c) zfma(acc, b.Up[i + (int64_t)c * b.r], x[b.SN[c]]);
      xr[i] = zsub(x[b.R[i]], acc);
    }
  } else {
    // Lp: nsn x r; output k = sum_i conj(Lp[i, k]) x[SN[i]]
    for (int k = wave; k < b.r; k += 4) {
      zd acc{0.0, 0.0};
      const zd* col = b.Lp + (int64_t)k * b.nsn;
      for (int i = lane; i < b.nsn; i += 64) zfmac(acc, col[i], x[b.SN[i]]);
      acc.re = wave_sum(acc.re);
      acc.im = wave_sum(acc.im);
      if (lane == 0) xr[k] = zsub(x[b.R[k]], acc);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < b.r; i += 256) x[b.R[i]] = xr[i];
  // x_S -= T x_R  (adjoint: conj(T) x_R); T: s x r, thread per row
  for (int l = threadIdx.x; l < b.s; l += 256) {
    zd d = gemv_n_row(b.T, b.s, l, b.r, xr, adjoint != 0);
    x[b.S[l]] = zsub(x[b.S[l]], d);
  }
}

__global__ void __launch_bounds__(256) gather_top_kernel(const int32_t* __restrict__ top, int n0,
                                                         const zd* __restrict__ x, zd* __restrict__ tmp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n0) tmp[i] = x[top[i]];
}

// x[top[i]] = sum_j Ainv[i, j] tmp[j]; thread per row
__global__ void __launch_bounds__(256) top_n_kernel(const zd* __restrict__ A, int n0,
                                                    const int32_t* __restrict__ top,
                                                    const zd* __restrict__ tmp, zd* __restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n0) return;
  zd acc{0.0, 0.0};
  for (int j = 0; j < n0; ++j) zfma(acc, A[i + (int64_t)j * n0], tmp[j]);
  x[top[i]] = acc;
}

// x[top[i]] = sum_j conj(Ainv[j, i]) tmp[j]; wave per output
__global__ void __launch_bounds__(256) top_c_kernel(const zd* __restrict__ A, int n0,
                                                    const int32_t* __restrict__ top,
                                                    const zd* __restrict__ tmp, zd* __restrict__ x) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= n0) return;
  zd d = gemv_t_wave(A, n0, i, n0, tmp, true, lane);
  if (lane == 0) x[top[i]] = d;
}

__global__ void __launch_bounds__(256) permute_kernel(const zd* __restrict__ src, zd* __restrict__ dst,
                                                      const int64_t* __restrict__ map, int64_t n,
                                                      int gather) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (gather)
    dst[i] = src[map[i]];
  else
    dst[map[i]] = src[i];
}

}  // namespace

void launch_solve_fwd(const SolveBox* boxes, int nb, int rmax, zd* x, zd* y, int adjoint,
                      hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(solve_fwd_kernel, dim3(nb), dim3(256), (size_t)rmax * sizeof(zd), st, boxes, x, y,
                     adjoint);
  FMMLU_HIP(hipGetLastError());
}

void launch_scatter_sub(const int32_t* dst, const int64_t* ptr, const int64_t* src, int64_t nd,
                        const zd* y, zd* x, hipStream_t st) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(scatter_sub_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, dst, ptr,
                     src, nd, y, x);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_diag(const SolveBox* boxes, int nb, int rmax, zd* x, int adjoint, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(solve_diag_kernel, dim3(nb), dim3(256), (size_t)rmax * sizeof(zd), st, boxes, x,
                     adjoint);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_bwd(const SolveBox* boxes, int nb, int rmax, zd* x, int adjoint, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(solve_bwd_kernel, dim3(nb), dim3(256), (size_t)rmax * sizeof(zd), st, boxes, x,
                     adjoint);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_top(const zd* Ainv, int n0, const int32_t* top, zd* x, zd* tmp, int adjoint,
                      hipStream_t st) {
  if (n0 <= 0) return;
  hipLaunchKernelGGL(gather_top_kernel, dim3((n0 + 255) / 256), dim3(256), 0, st, top, n0, x, tmp);
  FMMLU_HIP(hipGetLastError());
  if (!adjoint)
    hipLaunchKernelGGL(top_n_kernel, dim3((n0 + 255) / 256), dim3(256), 0, st, Ainv, n0, top, tmp, x);
  else
    hipLaunchKernelGGL(top_c_kernel, dim3((n0 + 3) / 4), dim3(256), 0, st, Ainv, n0, top, tmp, x);
  FMMLU_HIP(hipGetLastError());
}

void launch_permute(const zd* src, zd* dst, const int64_t* map, int64_t n, int gather,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, map,
                     n, gather);
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
