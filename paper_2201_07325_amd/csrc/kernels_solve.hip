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

// y[0:M] = op(A)[0:M, 0:K] v with A column-major (lda); v[k] = fetch(k). Lanes take rows,
// the four wavefronts split k, partial sums meet in LDS (part: 4 x 64). Result handed to
// emit(i, value) for i < M. Call from all 256 threads.
template <class FT, class Fetch, class Emit>
__device__ inline void block_gemv_n(const FT* __restrict__ A, int64_t lda, int M, int K, bool conjA,
                                    Fetch fetch, Emit emit, zd (*part)[64]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = 0; i0 < M; i0 += 64) {
    const int i = i0 + lane;
    zd acc{0.0, 0.0};
    if (i < M) {
      for (int k = wave; k < K; k += 4) {
        zd a = widen(A[i + (int64_t)k * lda]);
        if (conjA) a.im = -a.im;
        zfma(acc, a, fetch(k));
      }
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && i < M) {
      zd sum = zadd(zadd(part[0][lane], part[1][lane]), zadd(part[2][lane], part[3][lane]));
      emit(i, sum);
    }
    __syncthreads();
  }
}

// y[i] = sum_k A[k, i]^(*) v[k] for i < M; wavefront per output, lanes over k (coalesced).
template <class FT, class Fetch, class Emit>
__device__ inline void block_gemv_t(const FT* __restrict__ A, int64_t lda, int M, int K, bool conjA,
                                    Fetch fetch, Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = wave; i < M; i += 4) {
    zd acc{0.0, 0.0};
    const FT* col = A + (int64_t)i * lda;
    for (int k = lane; k < K; k += 64) {
      if (conjA)
        zfmac(acc, widen(col[k]), fetch(k));
      else
        zfma(acc, widen(col[k]), fetch(k));
    }
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) emit(i, acc);
  }
}

// Column GEMV partials: out[i] = sum_{k in [k0, k0+kn)} A[k, i]^(*) v[k] for the outputs of
// one group, four per wavefront at a time, lanes over k (coalesced down columns of A), v in
// LDS. kn <= kSolveK.
template <class FT, class Emit>
__device__ inline void colgemv_group(const FT* __restrict__ A, int64_t lda, int i0, int i1, int kn, bool conjA,
                                     const zd* v, Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int ib = i0 + 4 * wave; ib < i1; ib += 16) {
    zd acc[4] = {zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}};
    zd a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = lane + 64 * j;
        a[q][j] = (ib + q < i1 && k < kn) ? widen(A[(int64_t)(ib + q) * lda + k]) : zd{0.0, 0.0};
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = lane + 64 * j;
      const zd vk = k < kn ? v[k] : zd{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (conjA)
          zfmac(acc[q], a[q][j], vk);
        else
          zfma(acc[q], a[q][j], vk);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q].re = wave_sum(acc[q].re);
      acc[q].im = wave_sum(acc[q].im);
      if (lane == 0 && ib + q < i1) emit(ib + q, acc[q]);
    }
  }
}

// Row GEMV partial: sum_{k < kn} A[i, k]^(*) v[k] for one row i (thread per row; rows
// consecutive across threads, so each k is one coalesced load), eight loads in flight.
template <class FT>
__device__ inline zd rowgemv(const FT* __restrict__ A, int64_t lda, int i, int kn, bool conjA, const zd* v) {
  zd acc[4] = {zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}};
  const FT* ar = A + i;
  int k = 0;
  for (; k + 7 < kn; k += 8) {
    zd a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = widen(ar[(int64_t)(k + q) * lda]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (conjA)
        zfmac(acc[q & 3], a[q], v[k + q]);
      else
        zfma(acc[q & 3], a[q], v[k + q]);
    }
  }
  for (; k < kn; ++k) {
    const zd a = widen(ar[(int64_t)k * lda]);
    if (conjA)
      zfmac(acc[0], a, v[k]);
    else
      zfma(acc[0], a, v[k]);
  }
  return zadd(zadd(acc[0], acc[1]), zadd(acc[2], acc[3]));
}

// Forward: Pxr[c][i] = sum_{k in s-chunk c} op(T)[k, i] x_S[k] (T^T, adjoint T^H).
template <class FT>
__global__ void __launch_bounds__(256) solve_xr_part_kernel(const SolveBox* __restrict__ boxes,
                                                            const SweepTask* __restrict__ tasks,
                                                            const zd* __restrict__ x, zd* __restrict__ Pxr,
                                                            int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xs[kSolveK];
  for (int q = threadIdx.x; q < t.kn; q += 256) xs[q] = x[b.S[t.k0 + q]];
  __syncthreads();
  zd* out = Pxr + b.xrp_off + (int64_t)(t.k0 / kSolveK) * b.r;
  const int i0 = t.grp * kSolveOut, i1 = min(b.r, i0 + kSolveOut);
  colgemv_group(static_cast<const FT*>(b.T) + t.k0, b.s, i0, i1, t.kn, adjoint != 0, xs,
                [&](int i, zd d) { out[i] = d; });
}

// Forward, per box: x_R -= sum_c Pxr[c]; the result also goes to XR for the row GEMVs.
__global__ void __launch_bounds__(256) solve_xr_fin_kernel(const SolveBox* __restrict__ boxes, zd* x,
                                                           zd* __restrict__ XR, const zd* __restrict__ Pxr) {
  const SolveBox b = boxes[blockIdx.x];
  for (int i = threadIdx.x; i < b.r; i += 256) {
    zd v = x[b.R[i]];
    for (int c = 0; c < b.nks; ++c) v = zsub(v, Pxr[b.xrp_off + (int64_t)c * b.r + i]);
    x[b.R[i]] = v;
    XR[b.xr_off + i] = v;
  }
}

// Forward: Yp[c][i] = sum_{k in r-chunk c} P[i, k] x_R[k], P = Lp (adjoint: conj(U^T)).
template <class FT>
__global__ void __launch_bounds__(256) solve_y_part_kernel(const SolveBox* __restrict__ boxes,
                                                           const SweepTask* __restrict__ tasks,
                                                           const zd* __restrict__ XR, zd* __restrict__ Yp,
                                                           int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xr[kSolveKr];
  const int kb = t.chunk * kSolveKr, kn = min(kSolveKr, b.r - kb);
  for (int q = threadIdx.x; q < kn; q += 256) xr[q] = XR[b.xr_off + kb + q];
  __syncthreads();
  const FT* P = static_cast<const FT*>(adjoint ? b.UpT : b.Lp) + (int64_t)kb * b.nsn;
  zd* out = Yp + b.yp_off + (int64_t)t.chunk * b.nsn;
  const int i = t.k0 + threadIdx.x;
  if (i < t.k0 + t.kn) out[i] = rowgemv(P, b.nsn, i, kn, adjoint != 0, xr);
}

// Forward: y[i] = sum_c Yp[c][i] for the rows of one (box, row chunk).
__global__ void __launch_bounds__(256) solve_y_red_kernel(const SolveBox* __restrict__ boxes,
                                                          const SweepTask* __restrict__ tasks,
                                                          const zd* __restrict__ Yp, zd* __restrict__ y) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  const int i = t.k0 + threadIdx.x;
  if (i >= t.k0 + t.kn) return;
  zd v{0.0, 0.0};
  for (int c = 0; c < b.nkr; ++c) v = zadd(v, Yp[b.yp_off + (int64_t)c * b.nsn + i]);
  y[b.y_off + i] = v;
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

template <class FT>
__global__ void __launch_bounds__(256) solve_diag_kernel(const SolveBox* __restrict__ boxes, zd* x,
                                                         int adjoint) {
  const SolveBox b = boxes[blockIdx.x];
  extern __shared__ zd xr[];
  __shared__ zd part[4][64];
  for (int l = threadIdx.x; l < b.r; l += 256) xr[l] = x[b.R[l]];
  __syncthreads();
  if (!adjoint)
    block_gemv_n(static_cast<const FT*>(b.Xi), b.r, b.r, b.r, false, [&](int k) { return xr[k]; },
                 [&](int i, zd v) { x[b.R[i]] = v; }, part);
  else
    block_gemv_t(static_cast<const FT*>(b.Xi), b.r, b.r, b.r, true, [&](int k) { return xr[k]; },
                 [&](int i, zd v) { x[b.R[i]] = v; });
}

// Backward: Pbuf[c][i] = sum_{k in chunk c of S u N} Q[k, i] x_SN[k], Q = U^T (adjoint:
// conj(Lp)), stored (s+nN) x r; per (box, chunk, output group).
template <class FT>
__global__ void __launch_bounds__(256) solve_bpart_kernel(const SolveBox* __restrict__ boxes,
                                                          const SweepTask* __restrict__ tasks,
                                                          const zd* __restrict__ x, zd* __restrict__ Pbuf,
                                                          int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xsn[kSolveK];
  for (int q = threadIdx.x; q < t.kn; q += 256) xsn[q] = x[b.SN[t.k0 + q]];
  __syncthreads();
  zd* out = Pbuf + b.p_off + (int64_t)t.chunk * b.r;
  const FT* Q = static_cast<const FT*>(adjoint ? b.Lp : b.UpT) + t.k0;
  const int i0 = t.grp * kSolveOut, i1 = min(b.r, i0 + kSolveOut);
  colgemv_group(Q, b.nsn, i0, i1, t.kn, adjoint != 0, xsn, [&](int i, zd d) { out[i] = d; });
}

// Backward, per box: x_R -= sum_c Pbuf[c]; the result also goes to XR.
__global__ void __launch_bounds__(256) solve_bfin_kernel(const SolveBox* __restrict__ boxes,
                                                         const zd* __restrict__ Pbuf, zd* x, zd* __restrict__ XR) {
  const SolveBox b = boxes[blockIdx.x];
  for (int i = threadIdx.x; i < b.r; i += 256) {
    zd v = x[b.R[i]];
    for (int c = 0; c < b.nchunk; ++c) v = zsub(v, Pbuf[b.p_off + (int64_t)c * b.r + i]);
    x[b.R[i]] = v;
    XR[b.xr_off + i] = v;
  }
}

// Backward: Pt[c][l] = sum_{k in r-chunk c} op(T)[l, k] x_R[k] (T, adjoint conj(T)), T: s x r.
template <class FT>
__global__ void __launch_bounds__(256) solve_bt_part_kernel(const SolveBox* __restrict__ boxes,
                                                            const SweepTask* __restrict__ tasks,
                                                            const zd* __restrict__ XR, zd* __restrict__ Pt,
                                                            int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xr[kSolveKr];
  const int kb = t.chunk * kSolveKr, kn = min(kSolveKr, b.r - kb);
  for (int q = threadIdx.x; q < kn; q += 256) xr[q] = XR[b.xr_off + kb + q];
  __syncthreads();
  const FT* T = static_cast<const FT*>(b.T) + (int64_t)kb * b.s;
  zd* out = Pt + b.tp_off + (int64_t)t.chunk * b.s;
  const int l = t.k0 + threadIdx.x;
  if (l < t.k0 + t.kn) out[l] = rowgemv(T, b.s, l, kn, adjoint != 0, xr);
}

// Backward: x_S -= sum_c Pt[c] for the rows of one (box, s-row chunk).
__global__ void __launch_bounds__(256) solve_bt_fin_kernel(const SolveBox* __restrict__ boxes,
                                                           const SweepTask* __restrict__ tasks,
                                                           const zd* __restrict__ Pt, zd* x) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  const int l = t.k0 + threadIdx.x;
  if (l >= t.k0 + t.kn) return;
  zd v{0.0, 0.0};
  for (int c = 0; c < b.nkr; ++c) v = zadd(v, Pt[b.tp_off + (int64_t)c * b.s + l]);
  x[b.S[l]] = zsub(x[b.S[l]], v);
}

__global__ void __launch_bounds__(256) gather_top_kernel(const int32_t* __restrict__ top, int n0,
                                                         const zd* __restrict__ x, zd* __restrict__ tmp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n0) tmp[i] = x[top[i]];
}

// Top block, normal: partial[cb][i] = sum_{j in column block cb} Ainv[i, j] tmp[j]
// (grid: row blocks of 256 x column blocks of 256), then a finish pass sums the partials.
__global__ void __launch_bounds__(256) top_n_part_kernel(const zd* __restrict__ A, int n0,
                                                         const zd* __restrict__ tmp, zd* __restrict__ part) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * 256;
  __shared__ zd tv[256];
  const int jn = min(256, n0 - j0);
  if (threadIdx.x < jn) tv[threadIdx.x] = tmp[j0 + threadIdx.x];
  __syncthreads();
  if (i >= n0) return;
  zd acc{0.0, 0.0};
  for (int j = 0; j < jn; ++j) zfma(acc, A[i + (int64_t)(j0 + j) * n0], tv[j]);
  part[(int64_t)blockIdx.y * n0 + i] = acc;
}
__global__ void __launch_bounds__(256) top_n_fin_kernel(int n0, int nblk, const int32_t* __restrict__ top,
                                                        const zd* __restrict__ part, zd* __restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n0) return;
  zd acc{0.0, 0.0};
  for (int c = 0; c < nblk; ++c) acc = zadd(acc, part[(int64_t)c * n0 + i]);
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



#define FMMLU_FT_LAUNCH(kern, grid, lds, ...)                                      \
  do {                                                                              \
    if (f32)                                                                        \
      hipLaunchKernelGGL(kern<zf>, dim3(grid), dim3(256), lds, st, __VA_ARGS__);    \
    else                                                                            \
      hipLaunchKernelGGL(kern<zd>, dim3(grid), dim3(256), lds, st, __VA_ARGS__);    \
    FMMLU_HIP(hipGetLastError());                                                   \
  } while (0)

void launch_solve_xr_part(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* x, zd* Pxr, int adjoint,
                          bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(solve_xr_part_kernel, nt, 0, boxes, tasks, x, Pxr, adjoint);
}

void launch_solve_xr_fin(const SolveBox* boxes, int nb, zd* x, zd* XR, const zd* Pxr, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(solve_xr_fin_kernel, dim3(nb), dim3(256), 0, st, boxes, x, XR, Pxr);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_y_part(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XR, zd* Yp, int adjoint,
                         bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(solve_y_part_kernel, nt, 0, boxes, tasks, XR, Yp, adjoint);
}

void launch_solve_y_red(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* Yp, zd* y, hipStream_t st) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(solve_y_red_kernel, dim3(nt), dim3(256), 0, st, boxes, tasks, Yp, y);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_bpart(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* x, zd* Pbuf,
                        int adjoint, bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(solve_bpart_kernel, nt, 0, boxes, tasks, x, Pbuf, adjoint);
}

void launch_solve_bfin(const SolveBox* boxes, int nb, const zd* Pbuf, zd* x, zd* XR, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(solve_bfin_kernel, dim3(nb), dim3(256), 0, st, boxes, Pbuf, x, XR);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_bt_part(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XR, zd* Pt, int adjoint,
                          bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(solve_bt_part_kernel, nt, 0, boxes, tasks, XR, Pt, adjoint);
}

void launch_solve_bt_fin(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* Pt, zd* x, hipStream_t st) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(solve_bt_fin_kernel, dim3(nt), dim3(256), 0, st, boxes, tasks, Pt, x);
  FMMLU_HIP(hipGetLastError());
}

void launch_scatter_sub(const int32_t* dst, const int64_t* ptr, const int64_t* src, int64_t nd,
                        const zd* y, zd* x, hipStream_t st) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(scatter_sub_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, dst, ptr,
                     src, nd, y, x);
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_diag(const SolveBox* boxes, int nb, int rmax, zd* x, int adjoint, bool f32, hipStream_t st) {
  if (nb <= 0) return;
  const size_t lds = (size_t)rmax * sizeof(zd);
  if (f32)
    hipLaunchKernelGGL(solve_diag_kernel<zf>, dim3(nb), dim3(256), lds, st, boxes, x, adjoint);
  else
    hipLaunchKernelGGL(solve_diag_kernel<zd>, dim3(nb), dim3(256), lds, st, boxes, x, adjoint);
  FMMLU_HIP(hipGetLastError());
}



void launch_solve_top(const zd* Ainv, int n0, const int32_t* top, zd* x, zd* tmp, int adjoint,
                      hipStream_t st) {
  if (n0 <= 0) return;
  hipLaunchKernelGGL(gather_top_kernel, dim3((n0 + 255) / 256), dim3(256), 0, st, top, n0, x, tmp);
  FMMLU_HIP(hipGetLastError());
  if (!adjoint) {
    const int nblk = (n0 + 255) / 256;
    zd* part = tmp + n0;
    hipLaunchKernelGGL(top_n_part_kernel, dim3(nblk, nblk), dim3(256), 0, st, Ainv, n0, tmp, part);
    FMMLU_HIP(hipGetLastError());
    hipLaunchKernelGGL(top_n_fin_kernel, dim3(nblk), dim3(256), 0, st, n0, nblk, top, part, x);
  } else {
    hipLaunchKernelGGL(top_c_kernel, dim3((n0 + 3) / 4), dim3(256), 0, st, Ainv, n0, top, tmp, x);
  }
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
