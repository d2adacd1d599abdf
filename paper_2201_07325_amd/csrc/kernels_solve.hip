// Sweeps of the factored inverse (Section 4.2):
//   A^{-1} ~ (W_1^{-1} ... W_M^{-1}) P_t D^{-1} P_t^T (V_M^{-1} ... V_1^{-1}),
//   V_i^{-1} = L E P^T applied as  x_R -= T^T x_S ;  x_{S u N} -= L_{(S u N)} x_R,
//   W_i^{-1} = P F U   applied as  x_R -= U x_{S u N} ;  x_S -= T x_R,
// with L = X_{(S u N) R} X_RR^{-1} and U = X_RR^{-1} X_{R (S u N)}, and the conjugate
// transposes of the same factors for the adjoint. Boxes of one colour never touch, so a
// colour's boxes run concurrently; their L-updates to shared near DOFs are summed by a
// deterministic gather (scatter_sub) instead of atomics.
//
// Per colour phase and direction two or three launches: column products over chunks of the
// skeleton (or S u N) into partials of x_R; then items of 64 rows that each rebuild x_R from
// the partials while staging it in LDS and apply their rows of L or T (the four wavefronts of
// an item split the columns, no further partials); forward, the scatter. On phases with few
// boxes the column products take groups of 16 outputs and the row products items of 16 rows
// (every wavefront then takes every 16th column), so that more compute units share the phase.
// x_R of every box lives in one buffer between the forward sweep, the pivot blocks and the
// backward sweep.
//
// Every kernel works on a block of NR right-hand sides at once (NR = 1 or kSolveBlock):
// internal vectors are interleaved, entry i of right-hand side c at [i NR + c], so each
// factor entry is read once per block and used NR times. These kernels are HBM-bound in
// principle: every factor byte is read once per sweep and block.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

// v summed over the wavefront (the sum is complete in lane 0): DPP within rows of 16
// (quads, half-row and row mirrors), then across rows
template <int CTRL>
__device__ inline double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}
__device__ inline double wave_sum(double v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141>(v);  // row_half_mirror
  v = dpp_add<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Column GEMV partials for NR right-hand sides: out(i, c) = sum_{k < kn} A[k, i]^(*) v[k][c]
// for the outputs i of one group, four per wavefront at a time, lanes over k (coalesced down
// columns of A), v in LDS. kn <= kSolveK.
template <class FT, int NR, class Emit>
__device__ inline void colgemv_group(const FT* __restrict__ A, int64_t lda, int i0, int i1, int kn, bool conjA,
                                     const zd (*v)[NR], Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int ib = i0 + 4 * wave; ib < i1; ib += 16) {
    zd a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = lane + 64 * j;
        a[q][j] = (ib + q < i1 && k < kn) ? widen(A[(int64_t)(ib + q) * lda + k]) : zd{0.0, 0.0};
      }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      zd acc[4] = {zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}, zd{0.0, 0.0}};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = lane + 64 * j;
        const zd vk = k < kn ? v[k][c] : zd{0.0, 0.0};
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
        if (lane == 0 && ib + q < i1) emit(ib + q, c, acc[q]);
      }
    }
  }
}

// Forward: Pxr[c-chunk][i] = sum_{k in s-chunk} op(T)[k, i] x_S[k] (T^T, adjoint T^H), for the
// gsz outputs of group t.grp (gsz = 64, or 16 on phases with few work items).
template <class FT, int NR>
__global__ void __launch_bounds__(256) solve_xr_part_kernel(const SolveBox* __restrict__ boxes,
                                                            const SweepTask* __restrict__ tasks,
                                                            const zd* __restrict__ x, zd* __restrict__ Pxr,
                                                            int adjoint, int gsz) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xs[kSolveK][NR];
  for (int e = threadIdx.x; e < t.kn * NR; e += 256) xs[e / NR][e % NR] = x[(int64_t)b.S[t.k0 + e / NR] * NR + e % NR];
  __syncthreads();
  zd* out = Pxr + (b.xrp_off + (int64_t)(t.k0 / kSolveK) * b.r) * NR;
  const int i0 = t.grp * gsz, i1 = min(b.r, i0 + gsz);
  colgemv_group<FT, NR>(static_cast<const FT*>(b.T) + t.k0, b.s, i0, i1, t.kn, adjoint != 0, xs,
                        [&](int i, int c, zd d) { out[(int64_t)i * NR + c] = d; });
}

// Dot products of the rows [k0, k0 + 64) of a column-major matrix M (ld) with x_R staged in
// LDS in chunks of kSolveK, one row per lane, the four wavefronts taking every fourth column
// (four loads in flight each); acc holds this wavefront's share. stage(kb, kn) fills
// xr[0, kn) with x_R[kb, kb + kn) (all threads, before the barrier).
template <class FT, int NR, class Stage>
__device__ inline void rows_times_xr(const FT* __restrict__ M, int64_t ld, int r, int i, bool row, bool conjM,
                                     zd (*xr)[NR], zd (&acc)[NR], Stage stage) {
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = zd{0.0, 0.0};
  for (int kb = 0; kb < r; kb += kSolveK) {
    const int kn = min(kSolveK, r - kb);
    stage(kb, kn);
    __syncthreads();
    if (row) {
      const FT* col = M + i + (int64_t)kb * ld;
      int k = wave;
      for (; k + 12 < kn; k += 16) {
        zd a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = widen(col[(int64_t)(k + 4 * q) * ld]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < NR; ++c) {
            if (conjM)
              zfmac(acc[c], a[q], xr[k + 4 * q][c]);
            else
              zfma(acc[c], a[q], xr[k + 4 * q][c]);
          }
      }
      for (; k < kn; k += 4) {
        const zd a = widen(col[(int64_t)k * ld]);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          if (conjM)
            zfmac(acc[c], a, xr[k][c]);
          else
            zfma(acc[c], a, xr[k][c]);
        }
      }
    }
    __syncthreads();
  }
}

// the four wavefronts' sums of row `lane` side by side in LDS (xr reused; after the loop)
template <int NR>
__device__ inline void rows_reduce(zd (*xr)[NR], const zd (&acc)[NR]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NR; ++c) xr[wave * 64 + lane][c] = acc[c];
  __syncthreads();
}

// As rows_times_xr for items of 16 rows: lane l takes row l % 16 and, with the other lanes
// and wavefronts, every 16th column from l / 16 + 4 wave on (eight loads in flight each); the
// 16 partial sums of each row meet in LDS (rows16_sum).
template <class FT, int NR, class Stage>
__device__ inline void rows16_times_xr(const FT* __restrict__ M, int64_t ld, int r, int i, bool row, bool conjM,
                                       zd (*xr)[NR], zd (&acc)[NR], Stage stage) {
  const int kl = ((threadIdx.x & 63) >> 4) + 4 * (threadIdx.x >> 6);
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = zd{0.0, 0.0};
  for (int kb = 0; kb < r; kb += kSolveK) {
    const int kn = min(kSolveK, r - kb);
    stage(kb, kn);
    __syncthreads();
    if (row) {
      const FT* col = M + i + (int64_t)kb * ld;
      for (int k0 = kl; k0 < kn; k0 += 128) {
        zd a[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + 16 * q;
          a[q] = k < kn ? widen(col[(int64_t)k * ld]) : zd{0.0, 0.0};
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + 16 * q;
          if (k < kn) {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
              if (conjM)
                zfmac(acc[c], a[q], xr[k][c]);
              else
                zfma(acc[c], a[q], xr[k][c]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// the 16 partial sums of row `rho` (< 16) left by rows16_times_xr, in a fixed order (call
// after every thread has stored its acc to xr[threadIdx.x] and a barrier)
template <int NR>
__device__ inline zd rows16_sum(zd (*xr)[NR], int rho, int c) {
  zd v{0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 16; ++j) v = zadd(v, xr[(j >> 2) * 64 + (j & 3) * 16 + rho][c]);
  return v;
}

// Forward, per (box, 64 rows of S u N): x_R = x[R] - sum of the x_R partials, staged chunk by
// chunk (the item of rows 0..63 also keeps it in XRg); y = op(P) x_R for the item's rows,
// P = Lp (adjoint conj(Up^T)). A box with no S u N rows has one item without rows. RPI = 16:
// the same in items of 16 rows (phases with few boxes). direct: no two boxes of the phase
// share a row of S u N, so each row is subtracted from x[SN] here (x - y, as the scatter
// would) instead of going to y; the rows written are never the rows of R that items read.
template <class FT, int NR, int RPI>
__global__ void __launch_bounds__(256) solve_y_kernel(const SolveBox* __restrict__ boxes,
                                                      const SweepTask* __restrict__ tasks, zd* __restrict__ x,
                                                      const zd* __restrict__ Pxr, zd* __restrict__ XRg,
                                                      zd* __restrict__ y, int adjoint, int direct) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xr[kSolveK][NR];
  const int lane = threadIdx.x & 63;
  const int rho = RPI == 64 ? lane : (lane & 15);
  const int i = t.k0 + rho;
  const bool keep = t.k0 == 0;
  zd acc[NR];
  const FT* P = static_cast<const FT*>(adjoint ? b.UpT : b.Lp);
  auto stage = [&](int kb, int kn) {
    for (int e = threadIdx.x; e < kn * NR; e += 256) {
      const int k = e / NR, c = e % NR;
      zd v = x[(int64_t)b.R[kb + k] * NR + c];
      for (int ch = 0; ch < b.nks; ++ch)
        v = zsub(v, Pxr[(b.xrp_off + (int64_t)ch * b.r + kb + k) * NR + c]);
      xr[k][c] = v;
      if (keep) XRg[(b.dx_off + kb + k) * NR + c] = v;
    }
  };
  if constexpr (RPI == 64) {
    rows_times_xr<FT, NR>(P, b.nsn, b.r, i, lane < t.kn, adjoint != 0, xr, acc, stage);
    rows_reduce<NR>(xr, acc);
    if (threadIdx.x < 64 && lane < t.kn) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const zd v = zadd(zadd(xr[lane][c], xr[64 + lane][c]), zadd(xr[128 + lane][c], xr[192 + lane][c]));
        if (direct) {
          const int64_t xi = (int64_t)b.SN[i] * NR + c;
          x[xi] = zsub(x[xi], v);
        } else {
          y[(b.y_off + i) * NR + c] = v;
        }
      }
    }
  } else {
    rows16_times_xr<FT, NR>(P, b.nsn, b.r, i, rho < t.kn, adjoint != 0, xr, acc, stage);
    rows_reduce<NR>(xr, acc);
    if (threadIdx.x < 16 && rho < t.kn) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const zd v = rows16_sum<NR>(xr, rho, c);
        if (direct) {
          const int64_t xi = (int64_t)b.SN[i] * NR + c;
          x[xi] = zsub(x[xi], v);
        } else {
          y[(b.y_off + i) * NR + c] = v;
        }
      }
    }
  }
}

template <int NR>
__global__ void __launch_bounds__(256) scatter_sub_kernel(const int32_t* __restrict__ dst,
                                                          const int64_t* __restrict__ ptr,
                                                          const int64_t* __restrict__ src,
                                                          int64_t nd, const zd* __restrict__ y,
                                                          zd* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nd * NR) return;
  const int64_t d = e / NR;
  const int c = (int)(e % NR);
  zd acc{0.0, 0.0};
  for (int64_t q = ptr[d]; q < ptr[d + 1]; ++q) acc = zadd(acc, y[src[q] * NR + c]);
  const int64_t xi = (int64_t)dst[d] * NR + c;
  x[xi] = zsub(x[xi], acc);
}

// Diagonal: XRd = Xi XRg (adjoint Xi^H XRg), one (box, 64 outputs) item per workgroup, the
// box's x_R in dynamic LDS.
// Normal: lanes take rows, the four wavefronts split k, partial sums meet in LDS.
// Adjoint: one wavefront per output, lanes over k (columns of Xi are contiguous).
template <class FT, int NR>
__global__ void __launch_bounds__(256) solve_diag_kernel(const SolveBox* __restrict__ boxes,
                                                         const SweepTask* __restrict__ tasks, const zd* XRg,
                                                         zd* XRd, int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  extern __shared__ zd xr_flat[];
  zd(*xr)[NR] = reinterpret_cast<zd(*)[NR]>(xr_flat);
  __shared__ zd part[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const zd* xin = XRg + b.dx_off * NR;
  zd* x = XRd + b.dx_off * NR;
  for (int e = threadIdx.x; e < b.r * NR; e += 256) xr[e / NR][e % NR] = xin[e];
  __syncthreads();
  const FT* Xi = static_cast<const FT*>(b.Xi);
  const int r = b.r, i0 = t.k0, i1 = t.k0 + t.kn;
  if (!adjoint) {
    // the item's 64 rows, one per lane; the four wavefronts take every fourth column (four
    // loads in flight each) and meet in LDS
    const int i = i0 + lane;
    zd acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = zd{0.0, 0.0};
    if (i < i1) {
      const FT* row = Xi + i;
      int k = wave;
      for (; k + 12 < r; k += 16) {
        zd a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = widen(row[(int64_t)(k + 4 * q) * r]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < NR; ++c) zfma(acc[c], a[q], xr[k + 4 * q][c]);
      }
      for (; k < r; k += 4) {
        const zd a = widen(row[(int64_t)k * r]);
#pragma unroll
        for (int c = 0; c < NR; ++c) zfma(acc[c], a, xr[k][c]);
      }
    }
#pragma unroll 1
    for (int c = 0; c < NR; ++c) {
      part[wave][lane] = acc[c];
      __syncthreads();
      if (wave == 0 && i < i1)
        x[(int64_t)i * NR + c] = zadd(zadd(part[0][lane], part[1][lane]), zadd(part[2][lane], part[3][lane]));
      __syncthreads();
    }
  } else {
    for (int i = i0 + wave; i < i1; i += 4) {
      const FT* col = Xi + (int64_t)i * r;
      zd acc[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[c] = zd{0.0, 0.0};
      for (int k = lane; k < r; k += 64) {
        const zd a = widen(col[k]);
#pragma unroll
        for (int c = 0; c < NR; ++c) zfmac(acc[c], a, xr[k][c]);
      }
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        acc[c].re = wave_sum(acc[c].re);
        acc[c].im = wave_sum(acc[c].im);
        if (lane == 0) x[(int64_t)i * NR + c] = acc[c];
      }
    }
  }
}

// Backward: Pbuf[chunk][i] = sum_{k in chunk of S u N} Q[k, i] x_SN[k], Q = U^T (adjoint:
// conj(Lp)), stored (s+nN) x r; per (box, chunk, output group).
template <class FT, int NR>
__global__ void __launch_bounds__(256) solve_bpart_kernel(const SolveBox* __restrict__ boxes,
                                                          const SweepTask* __restrict__ tasks,
                                                          const zd* __restrict__ x, zd* __restrict__ Pbuf,
                                                          int adjoint, int gsz) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xsn[kSolveK][NR];
  for (int e = threadIdx.x; e < t.kn * NR; e += 256)
    xsn[e / NR][e % NR] = x[(int64_t)b.SN[t.k0 + e / NR] * NR + e % NR];
  __syncthreads();
  zd* out = Pbuf + (b.p_off + (int64_t)t.chunk * b.r) * NR;
  const FT* Q = static_cast<const FT*>(adjoint ? b.Lp : b.UpT) + t.k0;
  const int i0 = t.grp * gsz, i1 = min(b.r, i0 + gsz);
  colgemv_group<FT, NR>(Q, b.nsn, i0, i1, t.kn, adjoint != 0, xsn,
                        [&](int i, int c, zd d) { out[(int64_t)i * NR + c] = d; });
}

// Backward, per (box, 64 rows of S): x_R = XRd - sum of the backward partials, staged chunk by
// chunk (the item of rows 0..63 also writes it to x[R]); x_S -= op(T) x_R for the item's rows
// (T, adjoint conj(T)). A box with s = 0 has one item without rows. RPI = 16: items of 16
// rows.
template <class FT, int NR, int RPI>
__global__ void __launch_bounds__(256) solve_bt_kernel(const SolveBox* __restrict__ boxes,
                                                       const SweepTask* __restrict__ tasks,
                                                       const zd* __restrict__ XRd, const zd* __restrict__ Pbuf,
                                                       zd* __restrict__ x, int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd xr[kSolveK][NR];
  const int lane = threadIdx.x & 63;
  const int rho = RPI == 64 ? lane : (lane & 15);
  const int l = t.k0 + rho;
  const bool keep = t.k0 == 0;
  zd acc[NR];
  auto stage = [&](int kb, int kn) {
    for (int e = threadIdx.x; e < kn * NR; e += 256) {
      const int k = e / NR, c = e % NR;
      zd v = XRd[(b.dx_off + kb + k) * NR + c];
      for (int ch = 0; ch < b.nchunk; ++ch)
        v = zsub(v, Pbuf[(b.p_off + (int64_t)ch * b.r + kb + k) * NR + c]);
      xr[k][c] = v;
      if (keep) x[(int64_t)b.R[kb + k] * NR + c] = v;
    }
  };
  if constexpr (RPI == 64) {
    rows_times_xr<FT, NR>(static_cast<const FT*>(b.T), b.s, b.r, l, lane < t.kn, adjoint != 0, xr, acc, stage);
    rows_reduce<NR>(xr, acc);
    if (threadIdx.x < 64 && lane < t.kn) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const int64_t xi = (int64_t)b.S[l] * NR + c;
        x[xi] = zsub(x[xi], zadd(zadd(xr[lane][c], xr[64 + lane][c]), zadd(xr[128 + lane][c], xr[192 + lane][c])));
      }
    }
  } else {
    rows16_times_xr<FT, NR>(static_cast<const FT*>(b.T), b.s, b.r, l, rho < t.kn, adjoint != 0, xr, acc, stage);
    rows_reduce<NR>(xr, acc);
    if (threadIdx.x < 16 && rho < t.kn) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const int64_t xi = (int64_t)b.S[l] * NR + c;
        x[xi] = zsub(x[xi], rows16_sum<NR>(xr, rho, c));
      }
    }
  }
}

template <int NR>
__global__ void __launch_bounds__(256) gather_top_kernel(const int32_t* __restrict__ top, int n0,
                                                         const zd* __restrict__ x, zd* __restrict__ tmp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n0 * NR) tmp[e] = x[(int64_t)top[e / NR] * NR + e % NR];
}

// Top block, normal, in items of 64 rows x 256 columns: partial[cb][i] = sum over the column
// block cb of Ainv[i, j] tmp[j] (rows one per lane, the four wavefronts splitting the columns)
template <int NR>
__global__ void __launch_bounds__(256) top_rows_part_kernel(const zd* __restrict__ A, int n0,
                                                            const zd* __restrict__ tmp, zd* __restrict__ part) {
  __shared__ zd xr[kSolveK][NR];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 64 + lane;
  const int k0 = blockIdx.y * 256, kn = min(256, n0 - k0);
  zd acc[NR];
  rows_times_xr<zd, NR>(A + (int64_t)k0 * n0, n0, kn, i, i < n0, false, xr, acc, [&](int kb, int kc) {
    for (int e = threadIdx.x; e < kc * NR; e += 256) xr[e / NR][e % NR] = tmp[(int64_t)(k0 + kb) * NR + e];
  });
  rows_reduce<NR>(xr, acc);
  if (threadIdx.x < 64 && i < n0) {
#pragma unroll
    for (int c = 0; c < NR; ++c)
      part[((int64_t)blockIdx.y * n0 + i) * NR + c] =
          zadd(zadd(xr[lane][c], xr[64 + lane][c]), zadd(xr[128 + lane][c], xr[192 + lane][c]));
  }
}

template <int NR>
__global__ void __launch_bounds__(256) top_n_fin_kernel(int n0, int nblk, const int32_t* __restrict__ top,
                                                        const zd* __restrict__ part, zd* __restrict__ x) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n0 * NR) return;
  const int i = e / NR, c = e % NR;
  zd acc{0.0, 0.0};
  for (int cb = 0; cb < nblk; ++cb) acc = zadd(acc, part[((int64_t)cb * n0 + i) * NR + c]);
  x[(int64_t)top[i] * NR + c] = acc;
}

// x[top[i]] = sum_j conj(Ainv[j, i]) tmp[j]; wavefront per output, lanes over j
template <int NR>
__global__ void __launch_bounds__(256) top_c_kernel(const zd* __restrict__ A, int n0,
                                                    const int32_t* __restrict__ top,
                                                    const zd* __restrict__ tmp, zd* __restrict__ x) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= n0) return;
  const zd* col = A + (int64_t)i * n0;
  zd acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = zd{0.0, 0.0};
  for (int k = lane; k < n0; k += 64) {
    const zd a = col[k];
#pragma unroll
    for (int c = 0; c < NR; ++c) zfmac(acc[c], a, tmp[(int64_t)k * NR + c]);
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    acc[c].re = wave_sum(acc[c].re);
    acc[c].im = wave_sum(acc[c].im);
    if (lane == 0) x[(int64_t)top[i] * NR + c] = acc[c];
  }
}

// gather: dst[i NR + c] = src[map[i] + c ld] (c < m; zero for m <= c < NR)
// scatter: dst[map[i] + c ld] = src[i NR + c] (c < m)
template <int NR>
__global__ void __launch_bounds__(256) permute_kernel(const zd* __restrict__ src, zd* __restrict__ dst,
                                                      const int64_t* __restrict__ map, int64_t n, int64_t ld,
                                                      int m, int gather) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * NR) return;
  const int64_t i = e / NR;
  const int c = (int)(e % NR);
  if (gather)
    dst[e] = c < m ? src[map[i] + (int64_t)c * ld] : zd{0.0, 0.0};
  else if (c < m)
    dst[map[i] + (int64_t)c * ld] = src[e];
}

}  // namespace

#define FMMLU_NR_LAUNCH(kern, grid, lds, ...)                                      \
  do {                                                                              \
    if (nr == 1)                                                                    \
      hipLaunchKernelGGL(kern<1>, dim3(grid), dim3(256), lds, st, __VA_ARGS__);     \
    else if (nr == kSolveBlock)                                                     \
      hipLaunchKernelGGL(kern<kSolveBlock>, dim3(grid), dim3(256), lds, st, __VA_ARGS__); \
    else                                                                            \
      throw Error(FMMLU_EINVAL, "solve block of " + std::to_string(nr) + " columns"); \
    FMMLU_HIP(hipGetLastError());                                                   \
  } while (0)

#define FMMLU_FT_NR_LAUNCH(kern, grid, lds, ...)                                       \
  do {                                                                                  \
    if (nr != 1) throw Error(FMMLU_EINVAL, "single-vector sweep kernel with " + std::to_string(nr) + " columns"); \
    if (f32)                                                                            \
      hipLaunchKernelGGL((kern<zf, 1>), dim3(grid), dim3(256), lds, st, __VA_ARGS__);   \
    else                                                                                \
      hipLaunchKernelGGL((kern<zd, 1>), dim3(grid), dim3(256), lds, st, __VA_ARGS__);   \
    FMMLU_HIP(hipGetLastError());                                                       \
  } while (0)

#define FMMLU_FT_RPI_LAUNCH(kern, grid, ...)                                                          \
  do {                                                                                                 \
    if (nr != 1) throw Error(FMMLU_EINVAL, "single-vector sweep kernel with " + std::to_string(nr) + " columns"); \
    if (rows != 16 && rows != kSolveRows)                                                              \
      throw Error(FMMLU_EINVAL, "sweep items of " + std::to_string(rows) + " rows");                   \
    if (f32 && rows == 16)                                                                             \
      hipLaunchKernelGGL((kern<zf, 1, 16>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    else if (f32)                                                                                      \
      hipLaunchKernelGGL((kern<zf, 1, kSolveRows>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);        \
    else if (rows == 16)                                                                               \
      hipLaunchKernelGGL((kern<zd, 1, 16>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    else                                                                                               \
      hipLaunchKernelGGL((kern<zd, 1, kSolveRows>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);        \
    FMMLU_HIP(hipGetLastError());                                                                      \
  } while (0)

void launch_solve_xr_part(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pxr,
                          int adjoint, bool f32, hipStream_t st, int nr) {
  if (nt <= 0) return;
  if (gsz < 1 || gsz > kSolveOut) throw Error(FMMLU_EINVAL, "column-product group of " + std::to_string(gsz));
  FMMLU_FT_NR_LAUNCH(solve_xr_part_kernel, nt, 0, boxes, tasks, x, Pxr, adjoint, gsz);
}

void launch_solve_y(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, zd* x, const zd* Pxr,
                    zd* XRg, zd* y, int adjoint, int direct, bool f32, hipStream_t st, int nr) {
  if (nt <= 0) return;
  FMMLU_FT_RPI_LAUNCH(solve_y_kernel, nt, boxes, tasks, x, Pxr, XRg, y, adjoint, direct);
}

void launch_solve_bpart(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pbuf,
                        int adjoint, bool f32, hipStream_t st, int nr) {
  if (nt <= 0) return;
  if (gsz < 1 || gsz > kSolveOut) throw Error(FMMLU_EINVAL, "column-product group of " + std::to_string(gsz));
  FMMLU_FT_NR_LAUNCH(solve_bpart_kernel, nt, 0, boxes, tasks, x, Pbuf, adjoint, gsz);
}

void launch_solve_bt(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, const zd* XRd,
                     const zd* Pbuf, zd* x, int adjoint, bool f32, hipStream_t st, int nr) {
  if (nt <= 0) return;
  FMMLU_FT_RPI_LAUNCH(solve_bt_kernel, nt, boxes, tasks, XRd, Pbuf, x, adjoint);
}

void launch_scatter_sub(const int32_t* dst, const int64_t* ptr, const int64_t* src, int64_t nd,
                        const zd* y, zd* x, hipStream_t st, int nr) {
  if (nd <= 0) return;
  FMMLU_NR_LAUNCH(scatter_sub_kernel, (unsigned)((nd * nr + 255) / 256), 0, dst, ptr, src, nd, y, x);
}

void launch_solve_diag(const SolveBox* boxes, const SweepTask* tasks, int nt, int rmax, const zd* XRg, zd* XRd,
                       int adjoint, bool f32, hipStream_t st, int nr) {
  if (nt <= 0) return;
  const size_t lds = (size_t)rmax * nr * sizeof(zd);
  if (lds > 65536)
    throw Error(FMMLU_EINVAL, "redundant set of " + std::to_string(rmax) + " DOFs exceeds the diagonal step's LDS bound");
  FMMLU_FT_NR_LAUNCH(solve_diag_kernel, nt, lds, boxes, tasks, XRg, XRd, adjoint);
}

void launch_solve_top(const zd* Ainv, int n0, const int32_t* top, zd* x, zd* tmp, int adjoint,
                      hipStream_t st, int nr) {
  if (n0 <= 0) return;
  if (nr != 1) throw Error(FMMLU_EINVAL, "single-vector top-block step with " + std::to_string(nr) + " columns");
  hipLaunchKernelGGL(gather_top_kernel<1>, dim3((n0 + 255) / 256), dim3(256), 0, st, top, n0, x, tmp);
  if (!adjoint) {
    const int nblk = (n0 + 255) / 256;
    zd* part = tmp + (int64_t)n0;
    hipLaunchKernelGGL(top_rows_part_kernel<1>, dim3((n0 + 63) / 64, nblk), dim3(256), 0, st, Ainv, n0, tmp, part);
    hipLaunchKernelGGL(top_n_fin_kernel<1>, dim3((n0 + 255) / 256), dim3(256), 0, st, n0, nblk, top, part, x);
  } else {
    hipLaunchKernelGGL(top_c_kernel<1>, dim3((n0 + 3) / 4), dim3(256), 0, st, Ainv, n0, top, tmp, x);
  }
  FMMLU_HIP(hipGetLastError());
}

void launch_solve_top_gather(int n0, const int32_t* top, const zd* x, zd* tmp, hipStream_t st, int nr) {
  if (n0 <= 0) return;
  FMMLU_NR_LAUNCH(gather_top_kernel, (n0 * nr + 255) / 256, 0, top, n0, x, tmp);
}

void launch_solve_top_fin(int n0, const int32_t* top, const zd* part, zd* x, hipStream_t st, int nr) {
  if (n0 <= 0) return;
  const int nblk = (n0 + 255) / 256;
  FMMLU_NR_LAUNCH(top_n_fin_kernel, (n0 * nr + 255) / 256, 0, n0, nblk, top, part, x);
}

void launch_permute(const zd* src, zd* dst, const int64_t* map, int64_t n, int gather,
                    hipStream_t st, int nr, int64_t ld, int m) {
  if (n <= 0) return;
  if (m < 1 || m > nr) throw Error(FMMLU_EINVAL, "permute: active columns out of range");
  FMMLU_NR_LAUNCH(permute_kernel, (unsigned)((n * nr + 255) / 256), 0, src, dst, map, n, ld, m, gather);
}

}  // namespace fmmlu
