// Sweeps of the factored inverse (Section 4.2) for blocks of kSolveBlock right-hand sides on
// the matrix cores: every product of a stored factor with the block's vectors is a small
// complex GEMM, computed with v_mfma_f64_16x16x4f64 (float32 factors are widened as they are
// read). The block is interleaved as in the single-vector sweeps (entry i of right-hand side
// c at [i NB + c]), and the work items are the same: column products over chunks of the
// skeleton (or S u N) into partials of x_R, then items of rows that rebuild x_R from the
// partials while staging it in LDS and apply their rows of L or T (16 or 64 outputs or rows
// per item as in the single-vector sweeps; the backward rows of T always in items of 16, with
// x_R summed once per phase beforehand where those items would each re-read many partials).
//
// A workgroup of four wavefronts computes 64 outputs x kSolveBlock columns; wavefront w owns
// outputs 16 w .. 16 w + 15 as kSolveBlock / 16 blocks of 16 x 16 of D (complex: real and
// imaginary parts in separate accumulators, four real MFMAs per block and k-step of 4). Operand layout (16 x 16 x 4, float64):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16] in
// accumulator element r. The staged vectors (B) are read from LDS in chunks of kApplyK.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

constexpr int NB = kSolveBlock;  // right-hand sides per block
constexpr int NCB = NB / 16;     // 16-column MFMA blocks per wavefront
constexpr int KC = kApplyK;      // k-chunk staged in LDS
static_assert(NB % 16 == 0, "the block is a whole number of 16-column MFMA blocks");

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mma(double a, double b, dbl4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// complex D += op(a) b, op = identity or conjugate, with D = (cr, ci)
__device__ inline void cmma(dbl4& cr, dbl4& ci, zd a, zd b, bool conj) {
  const double ai = conj ? -a.im : a.im;
  cr = mma(a.re, b.re, cr);
  cr = mma(-ai, b.im, cr);
  ci = mma(a.re, b.im, ci);
  ci = mma(ai, b.re, ci);
}

// Accumulates this wavefront's 16 x NB block of D = sum_k op(A)[i, k] V[k, c] over
// k in [0, kn), V staged in sv[k][c], as NCB MFMA blocks of 16 columns. ROWS: A[i, k] =
// M[i + k ld] (rows i of a column-major matrix; the 16 lanes of a k-group read 16 consecutive
// rows); otherwise A[i, k] = M[i ld + k] (columns of the stored matrix, contiguous in k). i
// counts from the wavefront's first output; outputs at or past ni and k at or past kn
// contribute zero. With one column block, consecutive k-steps alternate between two
// accumulator sets (independent MFMA chains); with more, the blocks are the independent chains.
template <bool ROWS, class FT>
__device__ inline void block_mma(const FT* __restrict__ M, int64_t ld, int ni, int kn, bool conj,
                                 const zd (*sv)[NB], dbl4 (&cr)[2][NCB], dbl4 (&ci)[2][NCB]) {
  const int lane = threadIdx.x & 63, il = lane & 15, kq = lane >> 4;
  const bool iok = il < ni;
  const FT* base = ROWS ? M + il : M + (int64_t)il * ld;
  auto at = [&](int k) -> zd {
    if (!iok || k >= kn) return zd{0.0, 0.0};
    return widen(ROWS ? base[(int64_t)k * ld] : base[k]);
  };
  int ks = 0;
  for (; ks + 16 <= kn; ks += 16) {
    zd a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = at(ks + 4 * q + kq);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const zd b = sv[ks + 4 * q + kq][16 * cb + il];
        cmma(cr[NCB == 1 ? (q & 1) : 0][cb], ci[NCB == 1 ? (q & 1) : 0][cb], a[q], b, conj);
      }
  }
  for (; ks < kn; ks += 4) {
    const int k = ks + kq;
    const zd a = at(k);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const zd b = k < kn ? sv[k][16 * cb + il] : zd{0.0, 0.0};
      cmma(cr[0][cb], ci[0][cb], a, b, conj);
    }
  }
}

// D element r of column block cb of this lane: output row (lane / 16) + 4 r of the
// wavefront's block, column 16 cb + lane % 16
__device__ inline zd dval(const dbl4 (&cr)[2][NCB], const dbl4 (&ci)[2][NCB], int cb, int r) {
  return zd{cr[0][cb][r] + cr[1][cb][r], ci[0][cb][r] + ci[1][cb][r]};
}

// Rows [i0, i0 + ni) (ni <= 64) times a staged vector block over k in [0, K): chunks of KC
// filled by stage(kb, kn, sv) (all threads; rows k >= kn of the chunk are never read), then
// emit(row, c, value) for every output of the wavefront's rows.
template <class FT, class Stage, class Emit>
__device__ inline void rows_block(const FT* __restrict__ M, int64_t ld, int i0, int ni, int K, bool conj,
                                  zd (*sv)[NB], Stage stage, Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = 16 * wave;
  dbl4 cr[2][NCB], ci[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      cr[h][cb] = dbl4{0, 0, 0, 0};
      ci[h][cb] = dbl4{0, 0, 0, 0};
    }
  for (int kb = 0; kb < K; kb += KC) {
    const int kn = min(KC, K - kb);
    stage(kb, kn, sv);
    __syncthreads();
    if (wi < ni) block_mma<true, FT>(M + i0 + wi + (int64_t)kb * ld, ld, ni - wi, kn, conj, sv, cr, ci);
    __syncthreads();
  }
  if (wi < ni) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wi + (lane >> 4) + 4 * r;
        if (i < ni) emit(i0 + i, 16 * cb + (lane & 15), dval(cr, ci, cb, r));
      }
  }
}

// Outputs [i0, i0 + ni) of op(A)^T v with A[k, i] = M[i ld + k] over k in [k0, k1) (the
// stored matrix's columns i, contiguous in k), staged as in rows_block.
template <class FT, class Stage, class Emit>
__device__ inline void cols_block(const FT* __restrict__ M, int64_t ld, int i0, int ni, int k0, int k1, bool conj,
                                  zd (*sv)[NB], Stage stage, Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = 16 * wave;
  dbl4 cr[2][NCB], ci[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      cr[h][cb] = dbl4{0, 0, 0, 0};
      ci[h][cb] = dbl4{0, 0, 0, 0};
    }
  for (int kb = k0; kb < k1; kb += KC) {
    const int kn = min(KC, k1 - kb);
    stage(kb, kn, sv);
    __syncthreads();
    if (wi < ni) block_mma<false, FT>(M + (int64_t)(i0 + wi) * ld + kb, ld, ni - wi, kn, conj, sv, cr, ci);
    __syncthreads();
  }
  if (wi < ni) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wi + (lane >> 4) + 4 * r;
        if (i < ni) emit(i0 + i, 16 * cb + (lane & 15), dval(cr, ci, cb, r));
      }
  }
}

// The 16 x NB partial blocks of the four wavefronts (left in cr/ci) summed in LDS in
// wavefront order; emit(i0 + i, c, value) for i < ni (sv reused: 4 x 16 rows of NB).
template <class Emit>
__device__ inline void sum_waves16(const dbl4 (&cr)[2][NCB], const dbl4 (&ci)[2][NCB], int i0, int ni,
                                   zd (*sv)[NB], Emit emit) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) sv[16 * wave + (lane >> 4) + 4 * r][16 * cb + (lane & 15)] = dval(cr, ci, cb, r);
  __syncthreads();
  for (int e = threadIdx.x; e < ni * NB; e += 256) {
    const int i = e / NB, c = e % NB;
    emit(i0 + i, c, zadd(zadd(sv[i][c], sv[16 + i][c]), zadd(sv[32 + i][c], sv[48 + i][c])));
  }
}

// Rows [i0, i0 + ni) (ni <= 16) times the staged vector block over k in [0, K): the four
// wavefronts split every staged chunk of KC = 64 columns into four runs of 16 and their 16 x NB
// partial blocks are summed in LDS (wavefront order) at the end: four times the work items of
// rows_block for short row ranges (the skeleton rows of a box).
template <class FT, class Stage, class Emit>
__device__ inline void rows_block16(const FT* __restrict__ M, int64_t ld, int i0, int ni, int K, bool conj,
                                    zd (*sv)[NB], Stage stage, Emit emit) {
  static_assert(KC == 64, "four runs of 16 columns per staged chunk");
  const int wave = threadIdx.x >> 6;
  dbl4 cr[2][NCB], ci[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      cr[h][cb] = dbl4{0, 0, 0, 0};
      ci[h][cb] = dbl4{0, 0, 0, 0};
    }
  for (int kb = 0; kb < K; kb += KC) {
    const int kn = min(KC, K - kb);
    stage(kb, kn, sv);
    __syncthreads();
    const int k0 = 16 * wave, kw = min(16, kn - k0);
    if (ni > 0 && kw > 0) block_mma<true, FT>(M + i0 + (int64_t)(kb + k0) * ld, ld, ni, kw, conj, sv + k0, cr, ci);
    __syncthreads();
  }
  sum_waves16(cr, ci, i0, ni, sv, emit);
}

// Outputs [i0, i0 + ni) (ni <= 16) of cols_block: the four wavefronts split every staged chunk
// of KC = 64 into four runs of 16 and sum their partial blocks at the end (four times the
// work items of cols_block for phases with few boxes).
template <class FT, class Stage, class Emit>
__device__ inline void cols_block16(const FT* __restrict__ M, int64_t ld, int i0, int ni, int k0, int k1, bool conj,
                                    zd (*sv)[NB], Stage stage, Emit emit) {
  static_assert(KC == 64, "four runs of 16 columns per staged chunk");
  const int wave = threadIdx.x >> 6;
  dbl4 cr[2][NCB], ci[2][NCB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      cr[h][cb] = dbl4{0, 0, 0, 0};
      ci[h][cb] = dbl4{0, 0, 0, 0};
    }
  for (int kb = k0; kb < k1; kb += KC) {
    const int kn = min(KC, k1 - kb);
    stage(kb, kn, sv);
    __syncthreads();
    const int kw0 = 16 * wave, kw = min(16, kn - kw0);
    if (ni > 0 && kw > 0)
      block_mma<false, FT>(M + (int64_t)i0 * ld + kb + kw0, ld, ni, kw, conj, sv + kw0, cr, ci);
    __syncthreads();
  }
  sum_waves16(cr, ci, i0, ni, sv, emit);
}

// forward: Pxr[chunk][i] = sum_{k in the s-chunk} op(T)[k, i] x_S[k] (T^T, adjoint T^H), for
// the G outputs of group t.grp (G = 64, or 16 on phases with few work items)
template <class FT, int G>
__global__ void __launch_bounds__(256) blk_xr_part_kernel(const SolveBox* __restrict__ boxes,
                                                          const SweepTask* __restrict__ tasks,
                                                          const zd* __restrict__ x, zd* __restrict__ Pxr,
                                                          int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd sv[KC][NB];
  const int i0 = t.grp * G;
  zd* out = Pxr + (b.xrp_off + (int64_t)t.chunk * b.r) * NB;
  auto stage = [&](int kb, int kn, zd(*s)[NB]) {
    for (int e = threadIdx.x; e < kn * NB; e += 256) s[e / NB][e % NB] = x[(int64_t)b.S[kb + e / NB] * NB + e % NB];
  };
  auto emit = [&](int i, int c, zd v) { out[(int64_t)i * NB + c] = v; };
  if constexpr (G == 16)
    cols_block16<FT>(static_cast<const FT*>(b.T), b.s, i0, min(G, b.r - i0), t.k0, t.k0 + t.kn, adjoint != 0, sv,
                     stage, emit);
  else
    cols_block<FT>(static_cast<const FT*>(b.T), b.s, i0, min(G, b.r - i0), t.k0, t.k0 + t.kn, adjoint != 0, sv,
                   stage, emit);
}

// forward, per (box, RPI rows of S u N): x_R = x[R] - sum of the partials (kept in XRg by the
// item of the first rows), y = op(P) x_R (Lp, adjoint conj(Up^T)) for the item's rows
template <class FT, int RPI>
__global__ void __launch_bounds__(256) blk_y_kernel(const SolveBox* __restrict__ boxes,
                                                    const SweepTask* __restrict__ tasks, zd* __restrict__ x,
                                                    const zd* __restrict__ Pxr, zd* __restrict__ XRg,
                                                    zd* __restrict__ y, int adjoint, int direct) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd sv[KC][NB];
  const bool keep = t.k0 == 0;
  auto stage = [&](int kb, int kn, zd(*s)[NB]) {
    for (int e = threadIdx.x; e < kn * NB; e += 256) {
      const int k = e / NB, c = e % NB;
      zd v = x[(int64_t)b.R[kb + k] * NB + c];
      for (int ch = 0; ch < b.nks; ++ch) v = zsub(v, Pxr[(b.xrp_off + (int64_t)ch * b.r + kb + k) * NB + c]);
      s[k][c] = v;
      if (keep) XRg[(b.dx_off + kb + k) * NB + c] = v;
    }
  };
  auto emit = [&](int i, int c, zd v) {
    if (direct) {  // as in the single-vector sweep: the row goes straight into x[SN]
      const int64_t xi = (int64_t)b.SN[i] * NB + c;
      x[xi] = zsub(x[xi], v);
    } else {
      y[(b.y_off + i) * NB + c] = v;
    }
  };
  const FT* P = static_cast<const FT*>(adjoint ? b.UpT : b.Lp);
  if constexpr (RPI == 16)
    rows_block16<FT>(P, b.nsn, t.k0, t.kn, b.r, adjoint != 0, sv, stage, emit);
  else
    rows_block<FT>(P, b.nsn, t.k0, t.kn, b.r, adjoint != 0, sv, stage, emit);
}

// pivot blocks, per (box, 64 outputs): XRd = Xi XRg (adjoint Xi^H XRg)
template <class FT>
__global__ void __launch_bounds__(256) blk_diag_kernel(const SolveBox* __restrict__ boxes,
                                                       const SweepTask* __restrict__ tasks,
                                                       const zd* __restrict__ XRg, zd* __restrict__ XRd,
                                                       int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd sv[KC][NB];
  const zd* src = XRg + b.dx_off * NB;
  zd* dst = XRd + b.dx_off * NB;
  auto stage = [&](int kb, int kn, zd(*s)[NB]) {
    for (int e = threadIdx.x; e < kn * NB; e += 256) s[e / NB][e % NB] = src[(int64_t)kb * NB + e];
  };
  auto emit = [&](int i, int c, zd v) { dst[(int64_t)i * NB + c] = v; };
  if (!adjoint)
    rows_block<FT>(static_cast<const FT*>(b.Xi), b.r, t.k0, t.kn, b.r, false, sv, stage, emit);
  else
    cols_block<FT>(static_cast<const FT*>(b.Xi), b.r, t.k0, t.kn, 0, b.r, true, sv, stage, emit);
}

// backward: Pb[chunk][i] = sum_{k in the chunk of S u N} op(Q)[k, i] x_SN[k] (U^T, adjoint
// conj(Lp)), output groups of G as in blk_xr_part_kernel
template <class FT, int G>
__global__ void __launch_bounds__(256) blk_bpart_kernel(const SolveBox* __restrict__ boxes,
                                                        const SweepTask* __restrict__ tasks,
                                                        const zd* __restrict__ x, zd* __restrict__ Pb, int adjoint) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd sv[KC][NB];
  const int i0 = t.grp * G;
  zd* out = Pb + (b.p_off + (int64_t)t.chunk * b.r) * NB;
  auto stage = [&](int kb, int kn, zd(*s)[NB]) {
    for (int e = threadIdx.x; e < kn * NB; e += 256) s[e / NB][e % NB] = x[(int64_t)b.SN[kb + e / NB] * NB + e % NB];
  };
  auto emit = [&](int i, int c, zd v) { out[(int64_t)i * NB + c] = v; };
  const FT* Q = static_cast<const FT*>(adjoint ? b.Lp : b.UpT);
  if constexpr (G == 16)
    cols_block16<FT>(Q, b.nsn, i0, min(G, b.r - i0), t.k0, t.k0 + t.kn, adjoint != 0, sv, stage, emit);
  else
    cols_block<FT>(Q, b.nsn, i0, min(G, b.r - i0), t.k0, t.k0 + t.kn, adjoint != 0, sv, stage, emit);
}

// backward, per (box, 64 entries of R): x_R = XRd - sum of the partials, stored back to XRd
// and to x[R] (phases whose row items would each re-read many partials)
__global__ void __launch_bounds__(256) blk_xr_sub_kernel(const SolveBox* __restrict__ boxes,
                                                         const SweepTask* __restrict__ tasks, zd* __restrict__ XRd,
                                                         const zd* __restrict__ Pb, zd* __restrict__ x) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  for (int e = threadIdx.x; e < t.kn * NB; e += 256) {
    const int k = t.k0 + e / NB, c = e % NB;
    zd v = XRd[(b.dx_off + k) * NB + c];
    for (int ch = 0; ch < b.nchunk; ++ch) v = zsub(v, Pb[(b.p_off + (int64_t)ch * b.r + k) * NB + c]);
    XRd[(b.dx_off + k) * NB + c] = v;
    x[(int64_t)b.R[k] * NB + c] = v;
  }
}

// backward, per (box, 16 rows of S): x_R = XRd - sum of the partials (written to x[R] by the
// item of rows 0..15), x_S -= op(T) x_R (T, adjoint conj(T)) for the item's rows. presummed:
// blk_xr_sub_kernel has already done the first step (x_R is XRd).
template <class FT>
__global__ void __launch_bounds__(256) blk_bt_kernel(const SolveBox* __restrict__ boxes,
                                                     const SweepTask* __restrict__ tasks, const zd* __restrict__ XRd,
                                                     const zd* __restrict__ Pb, zd* __restrict__ x, int adjoint,
                                                     int presummed) {
  const SweepTask t = tasks[blockIdx.x];
  const SolveBox b = boxes[t.box];
  __shared__ zd sv[KC][NB];
  const bool keep = t.k0 == 0 && !presummed;
  const int nch = presummed ? 0 : b.nchunk;
  rows_block16<FT>(static_cast<const FT*>(b.T), b.s, t.k0, t.kn, b.r, adjoint != 0, sv,
                 [&](int kb, int kn, zd(*s)[NB]) {
                   for (int e = threadIdx.x; e < kn * NB; e += 256) {
                     const int k = e / NB, c = e % NB;
                     zd v = XRd[(b.dx_off + kb + k) * NB + c];
                     for (int ch = 0; ch < nch; ++ch)
                       v = zsub(v, Pb[(b.p_off + (int64_t)ch * b.r + kb + k) * NB + c]);
                     s[k][c] = v;
                     if (keep) x[(int64_t)b.R[kb + k] * NB + c] = v;
                   }
                 },
                 [&](int l, int c, zd v) {
                   const int64_t xi = (int64_t)b.S[l] * NB + c;
                   x[xi] = zsub(x[xi], v);
                 });
}

// top block partials: part[kc][i] = sum_{j in chunk kc} Ainv[i, j] tmp[j] (adjoint
// conj(Ainv[j, i])), grid (64-output blocks) x (chunks of 256)
__global__ void __launch_bounds__(256) blk_top_part_kernel(const zd* __restrict__ A, int n0,
                                                           const zd* __restrict__ tmp, zd* __restrict__ part,
                                                           int adjoint) {
  __shared__ zd sv[KC][NB];
  const int i0 = blockIdx.x * 64, ni = min(64, n0 - i0);
  const int k0 = blockIdx.y * 256, k1 = min(n0, k0 + 256);
  zd* out = part + (int64_t)blockIdx.y * n0 * NB;
  auto stage = [&](int kb, int kn, zd(*s)[NB]) {
    for (int e = threadIdx.x; e < kn * NB; e += 256) s[e / NB][e % NB] = tmp[(int64_t)kb * NB + e];
  };
  auto emit = [&](int i, int c, zd v) { out[(int64_t)i * NB + c] = v; };
  if (!adjoint) {
    rows_block<zd>(A + (int64_t)k0 * n0, n0, i0, ni, k1 - k0, false, sv,
                   [&](int kb, int kn, zd(*s)[NB]) { stage(k0 + kb, kn, s); }, emit);
  } else {
    cols_block<zd>(A, n0, i0, ni, k0, k1, true, sv, stage, emit);
  }
}

}  // namespace

#define FMMLU_FT_LAUNCH(kern, grid, ...)                                               \
  do {                                                                                  \
    if (f32)                                                                            \
      hipLaunchKernelGGL(kern<zf>, dim3(grid), dim3(256), 0, st, __VA_ARGS__);          \
    else                                                                                \
      hipLaunchKernelGGL(kern<zd>, dim3(grid), dim3(256), 0, st, __VA_ARGS__);          \
    FMMLU_HIP(hipGetLastError());                                                       \
  } while (0)

// kern<FT, 16> or kern<FT, 64> by the granularity g (outputs or rows per work item)
#define FMMLU_FT_G_LAUNCH(kern, grid, g, ...)                                                        \
  do {                                                                                              \
    if (g != 16 && g != 64) throw Error(FMMLU_EINVAL, "blocked sweep items of " + std::to_string(g)); \
    if (f32 && g == 16)                                                                             \
      hipLaunchKernelGGL((kern<zf, 16>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    else if (f32)                                                                                   \
      hipLaunchKernelGGL((kern<zf, 64>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    else if (g == 16)                                                                               \
      hipLaunchKernelGGL((kern<zd, 16>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    else                                                                                            \
      hipLaunchKernelGGL((kern<zd, 64>), dim3(grid), dim3(256), 0, st, __VA_ARGS__);                \
    FMMLU_HIP(hipGetLastError());                                                                   \
  } while (0)

void launch_blk_xr_part(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pxr,
                        int adjoint, bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_G_LAUNCH(blk_xr_part_kernel, nt, gsz, boxes, tasks, x, Pxr, adjoint);
}

void launch_blk_y(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, zd* x, const zd* Pxr,
                  zd* XRg, zd* y, int adjoint, int direct, bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_G_LAUNCH(blk_y_kernel, nt, rows, boxes, tasks, x, Pxr, XRg, y, adjoint, direct);
}

void launch_blk_diag(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XRg, zd* XRd, int adjoint,
                     bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(blk_diag_kernel, nt, boxes, tasks, XRg, XRd, adjoint);
}

void launch_blk_bpart(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pb,
                      int adjoint, bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_G_LAUNCH(blk_bpart_kernel, nt, gsz, boxes, tasks, x, Pb, adjoint);
}

void launch_blk_xr_sub(const SolveBox* boxes, const SweepTask* tasks, int nt, zd* XRd, const zd* Pb, zd* x,
                       hipStream_t st) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(blk_xr_sub_kernel, dim3(nt), dim3(256), 0, st, boxes, tasks, XRd, Pb, x);
  FMMLU_HIP(hipGetLastError());
}

void launch_blk_bt(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XRd, const zd* Pb, zd* x,
                   int adjoint, int presummed, bool f32, hipStream_t st) {
  if (nt <= 0) return;
  FMMLU_FT_LAUNCH(blk_bt_kernel, nt, boxes, tasks, XRd, Pb, x, adjoint, presummed);
}

void launch_blk_top_part(const zd* Ainv, int n0, const zd* tmp, zd* part, int adjoint, hipStream_t st) {
  if (n0 <= 0) return;
  const dim3 grid((unsigned)((n0 + 63) / 64), (unsigned)((n0 + 255) / 256));
  hipLaunchKernelGGL(blk_top_part_kernel, grid, dim3(256), 0, st, Ainv, n0, tmp, part, adjoint);
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
