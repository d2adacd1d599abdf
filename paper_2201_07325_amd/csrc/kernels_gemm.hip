// Batched complex GEMM on the matrix cores. Operands A and B are complex float64 in memory.
// The register-staged kernels compute in float64 (v_mfma_f64_16x16x4f64) for float64 C and
// in float32 (v_mfma_f32_16x16x4f32, operands rounded as they are staged) for float32 C; the
// direct-to-LDS kernel always computes in float64 and rounds a float32 C as it stores it.
//
//   C[rmap[i], cmap[j]] = beta C[...] + alpha * sum_s opA(A_s)[i, :] B_s[:, j]
//
// A workgroup of four wavefronts computes a 64 x 64 block of C; each wavefront owns a
// 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16, with the real and imaginary parts
// accumulated separately: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br (four real MFMAs per
// complex block and k-step of 4). K is staged through LDS in steps of 16, as separate real
// and imaginary planes; for float32 with eight wavefronts the global loads run two steps ahead
// of the step in LDS (two register sets used in turn), so each load has two steps of the
// shorter float32 MFMAs to arrive (one step ahead otherwise). MFMA operand layout (16 x 16 x
// 4, float64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[l / 16 + 4 r][l % 16] (float64) or D[4 (l / 16) + r][l % 16]
// (float32) in accumulator element r.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <class CT>
struct Mfma;
template <>
struct Mfma<zd> {
  using R = double;
  using V = dbl4;
  __device__ static V mma(R a, R b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<zf> {
  using R = float;
  using V = flt4;
  __device__ static V mma(R a, R b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class Task>
__device__ inline int find_unit_task(const Task* __restrict__ t, int n, int64_t u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].unit_begin <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr int BM = kGemmTile, BN = kGemmTile, BK = 16;
constexpr int LDP = BM + 4;  // padded LDS row (doubles)

// SCAT: C entries through the row / column maps (the Schur updates of pair tiles)
// NWV wavefronts per workgroup (4: each owns a 32 x 32 quarter of the 64 x 64 block; 8: a
// 32 x 16 eighth, with half the accumulators and staging registers, so more wavefronts
// fit per SIMD)
template <int OPA, class CT, bool SCAT, int NWV>
__global__ void __launch_bounds__(64 * NWV, NWV == 8 ? 4 : 3)
    zgemm_mfma_kernel(const GemmTask* __restrict__ tasks, int ntasks, const GemmSeg* __restrict__ segs,
                      const int32_t* __restrict__ utask) {
  constexpr int GT = 64 * NWV;          // threads
  constexpr int NQ = BM * BK / GT;      // staged values per thread and operand per K step
  constexpr int WB = 8 / NWV;           // 16-column blocks per wavefront
  using M = Mfma<CT>;
  using R = typename M::R;
  __shared__ R Asr[BK][LDP], Asi[BK][LDP], Bsr[BK][LDP], Bsi[BK][LDP];
  // blocks are dealt to the 8 XCDs in turn: in each round of 64 blocks, XCD x gets the 8
  // consecutive output blocks 8x .. 8x + 7 (neighbouring tiles of a task share its panels
  // in that XCD's L2); the last partial round keeps the identity
  int64_t u = blockIdx.x;
  {
    const int64_t g = gridDim.x, full = g - g % 64;
    if (u < full) u = (u & ~int64_t(63)) + (u & 7) * 8 + ((u >> 3) & 7);
  }
  const GemmTask t = tasks[utask ? utask[u] : find_unit_task(tasks, ntasks, u)];
  if (t.skip && *t.skip) return;
  int64_t lu = u - t.unit_begin;
  const int nbm = (t.M + BM - 1) / BM;
  const int64_t ntiles = gemm_task_tiles(t.M, t.N, t.lower);
  const int kc = (int)(lu / ntiles);  // split-K chunk (0 without split)
  lu -= (int64_t)kc * ntiles;
  int row0, col0;
  if (t.lower) {
    // lu = ti (ti + 1) / 2 + tj with tj <= ti
    int ti = (int)((sqrt(8.0 * (double)lu + 1.0) - 1.0) * 0.5);
    while ((int64_t)(ti + 1) * (ti + 2) / 2 <= lu) ++ti;
    while ((int64_t)ti * (ti + 1) / 2 > lu) --ti;
    row0 = ti * BM;
    col0 = (int)(lu - (int64_t)ti * (ti + 1) / 2) * BN;
  } else {
    row0 = (int)(lu % nbm) * BM;
    col0 = (int)(lu / nbm) * BN;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 16 * WB;  // wavefront's 32 x 16 WB part
  // 16 x 16 blocks of the part that hold entries of C (wave-uniform): the others skip
  // their MFMAs and operand reads
  const int vm = t.M - row0 - wr, vn = t.N - col0 - wc;
  bool ua[2] = {vm > 0, vm > 16}, ub[WB];
#pragma unroll
  for (int b = 0; b < WB; ++b) ub[b] = vn > 16 * b;
  typename M::V cr[2][WB], ci[2][WB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b) {
      cr[a][b] = typename M::V{0, 0, 0, 0};
      ci[a][b] = typename M::V{0, 0, 0, 0};
    }
  // the K steps of all segments form one stream: the global loads of the next step (which
  // may belong to the next segment) are issued before the current step's products
  auto krange = [&](const GemmSeg& g, int& b, int& e) {
    b = t.kchunk > 0 ? kc * t.kchunk : 0;
    e = t.kchunk > 0 ? min(g.K, b + t.kchunk) : g.K;
  };
  // first segment with work at or after index s (t.nseg if none)
  auto next_seg = [&](int s, GemmSeg& g, int& b, int& e) {
    for (; s < t.nseg; ++s) {
      g = segs[t.seg_begin + s];
      krange(g, b, e);
      if (b < e) break;
    }
    return s;
  };
  // global values of the two steps ahead of the one in LDS (two register sets, used in turn)
  zd ra0[NQ], rb0[NQ], ra1[NQ], rb1[NQ];
  auto load = [&](zd(&ra)[NQ], zd(&rb)[NQ], const GemmSeg& sg, int k0, int kend) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + GT * q;
      int i, kk;
      if (OPA == 0) {
        i = e % BM;
        kk = e / BM;
      } else {
        kk = e % BK;
        i = e / BK;
      }
      const int gi = row0 + i, gk = k0 + kk;
      zd v{0.0, 0.0};
      if (gi < t.M && gk < kend) {
        if (OPA == 0) {
          v = sg.A[gi + (int64_t)gk * sg.lda];
          if (sg.ishift > 0 && gi == sg.ishift - 1 + gk) v.re -= 1.0;
        } else {
          v = sg.A[gk + (int64_t)gi * sg.lda];
          if (OPA == 2) v.im = -v.im;
        }
      }
      ra[q] = v;
      const int kb = e % BK, j = e / BK;
      const int gkb = k0 + kb, gj = col0 + j;
      zd w{0.0, 0.0};
      if (gkb < kend && gj < t.N) w = sg.B[gkb + (int64_t)gj * sg.ldb];
      rb[q] = w;
    }
  };
  auto store = [&](const zd(&ra)[NQ], const zd(&rb)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + GT * q;
      int i, kk;
      if (OPA == 0) {
        i = e % BM;
        kk = e / BM;
      } else {
        kk = e % BK;
        i = e / BK;
      }
      Asr[kk][i] = (R)ra[q].re;
      Asi[kk][i] = (R)ra[q].im;
      const int kb = e % BK, j = e / BK;
      Bsr[kb][j] = (R)rb[q].re;
      Bsi[kb][j] = (R)rb[q].im;
    }
  };
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      R ar[2], ai[2], an[2], br[WB], bi[WB];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = ua[a] ? Asr[kr][wr + 16 * a + cl] : R(0);
        ai[a] = ua[a] ? Asi[kr][wr + 16 * a + cl] : R(0);
        an[a] = -ai[a];
      }
#pragma unroll
      for (int b = 0; b < WB; ++b) {
        br[b] = ub[b] ? Bsr[kr][wc + 16 * b + cl] : R(0);
        bi[b] = ub[b] ? Bsi[kr][wc + 16 * b + cl] : R(0);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          if (!(ua[a] && ub[b])) continue;
          cr[a][b] = M::mma(ar[a], br[b], cr[a][b]);
          cr[a][b] = M::mma(an[a], bi[b], cr[a][b]);
          ci[a][b] = M::mma(ar[a], bi[b], ci[a][b]);
          ci[a][b] = M::mma(ai[a], br[b], ci[a][b]);
        }
    }
  };
  if constexpr (NWV == 4 || sizeof(R) == 8) {
    // four wavefronts hold twice the accumulators, and a float64 MFMA step is long enough to
    // cover the loads: one register set, loads one step ahead (a second set would cost one of
    // the six wavefronts per SIMD)
    GemmSeg cur;
    int kb0, ke0;
    int cs = next_seg(0, cur, kb0, ke0);
    int ck = kb0;
    if (cs < t.nseg) load(ra0, rb0, cur, ck, ke0);
    while (cs < t.nseg) {
      // position of the next step
      GemmSeg nxt = cur;
      int ns = cs, nk = ck + BK, ne = ke0;
      if (nk >= ke0) ns = next_seg(cs + 1, nxt, nk, ne);
      __syncthreads();
      store(ra0, rb0);
      __syncthreads();
      if (ns < t.nseg) load(ra0, rb0, nxt, nk, ne);
      compute();
      cs = ns;
      ck = nk;
      ke0 = ne;
      cur = nxt;
    }
  } else {
    // total K steps over the segments; the load cursor runs two steps ahead of the LDS copy
    int nsteps = 0;
    for (int q = 0; q < t.nseg; ++q) {
      int b, e;
      krange(segs[t.seg_begin + q], b, e);
      if (b < e) nsteps += (e - b + BK - 1) / BK;
    }
    GemmSeg lg;
    int lk, le;
    int ls = next_seg(0, lg, lk, le);
    auto advance = [&]() {
      lk += BK;
      if (lk >= le) ls = next_seg(ls + 1, lg, lk, le);
    };
    if (nsteps > 0) {
      load(ra0, rb0, lg, lk, le);
      advance();
    }
    if (nsteps > 1) {
      load(ra1, rb1, lg, lk, le);
      advance();
    }
    for (int st = 0; st < nsteps; st += 2) {
      __syncthreads();
      store(ra0, rb0);
      __syncthreads();
      if (st + 2 < nsteps) {
        load(ra0, rb0, lg, lk, le);
        advance();
      }
      compute();
      if (st + 1 >= nsteps) break;
      __syncthreads();
      store(ra1, rb1);
      __syncthreads();
      if (st + 3 < nsteps) {
        load(ra1, rb1, lg, lk, le);
        advance();
      }
      compute();
    }
  }
  const zd alpha{t.alpha_re, t.alpha_im};
  CT* Cb = static_cast<CT*>(t.C) + (int64_t)kc * t.part_stride;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + wr + 16 * a + M::row(lane, r);
        const int j = col0 + wc + 16 * b + (lane & 15);
        if (i >= t.M || j >= t.N) continue;
        const int ri = (SCAT && t.rmap) ? t.rmap[i] : i;
        const int cj = (SCAT && t.cmap) ? t.cmap[j] : j;
        CT* c = Cb + ri + (int64_t)cj * t.ldc;
        zd v = zmul(alpha, zd{(double)cr[a][b][r], (double)ci[a][b][r]});
        if (t.beta != 0.0) v = zadd(v, zscale(widen(*c), t.beta));
        *c = narrow<CT>(v);
      }
}

// ---------------------------------------------------------------------------------------
// The same batched GEMM for opA = N with float64 C, operands copied from global memory
// straight into LDS (global_load_lds_dwordx4: no staging registers), two LDS buffers used in
// turn, one barrier per K step. TM x TM output blocks (instantiated for TM = 64): eight
// wavefronts in a 2 x 4 grid, each owning a (TM / 2) x (TM / 4) part. Per buffer: A as [16 k][TM rows] and B
// as [TM cols][16 k] of interleaved complex values; within a B column the 16 k positions are
// XOR-swizzled with the column's low four bits, so that the 16 lanes of an MFMA operand read
// (16 columns, one k) fall into 16 different LDS bank groups. Loads outside the task are
// clamped to its last row, column or k (finite values): rows and columns outside C are never
// stored, and k positions past the segment's end are zeroed in the A operand. A segment's
// shifted identity (ishift, unmapped launches only) is subtracted as the A operand is read from
// LDS. LDS: 64 KB per workgroup (TM = 64), dynamic, so two workgroups share a compute unit.
// (128 x 128 blocks, one workgroup per compute unit, measured slower on the Schur updates:
// 37.6 vs 29.4 ms.) The output rows and columns are read through the maps before the K loop,
// and the epilogue issues all old values of C before its stores.
template <int OPA, bool SCAT, int TM, class CT = zd>
__global__ void __launch_bounds__(512, TM == 64 ? 4 : 2)
    zgemm_lds_kernel(const GemmTask* __restrict__ tasks, int ntasks, const GemmSeg* __restrict__ segs,
                     const int32_t* __restrict__ utask) {
  using M = Mfma<zd>;
  constexpr int AB = TM / 32, BB = TM / 64;  // 16 x 16 MFMA blocks per wavefront: rows, columns
  constexpr int NLA = TM / 32;               // LDS copies per wavefront and operand per K step
  extern __shared__ __align__(16) unsigned char smem_raw[];
  zd* lds = reinterpret_cast<zd*>(smem_raw);  // [buffer][A: 16 TM | B: TM 16]
  int64_t u = blockIdx.x;
  {
    const int64_t g = gridDim.x, full = g - g % 64;
    if (u < full) u = (u & ~int64_t(63)) + (u & 7) * 8 + ((u >> 3) & 7);
  }
  const GemmTask t = tasks[utask ? utask[u] : find_unit_task(tasks, ntasks, u)];
  if (t.skip && *t.skip) return;
  int64_t lu = u - t.unit_begin;
  const int nbm = (t.M + TM - 1) / TM;
  const int64_t ntiles = gemm_task_tiles_t(t.M, t.N, t.lower, TM);
  const int kc = (int)(lu / ntiles);
  lu -= (int64_t)kc * ntiles;
  int row0, col0;
  if (t.lower) {
    int ti = (int)((sqrt(8.0 * (double)lu + 1.0) - 1.0) * 0.5);
    while ((int64_t)(ti + 1) * (ti + 2) / 2 <= lu) ++ti;
    while ((int64_t)ti * (ti + 1) / 2 > lu) --ti;
    row0 = ti * TM;
    col0 = (int)(lu - (int64_t)ti * (ti + 1) / 2) * TM;
  } else {
    row0 = (int)(lu % nbm) * TM;
    col0 = (int)(lu / nbm) * TM;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * (TM / 2), wc = (wave >> 1) * (TM / 4);  // wavefront's part
  const int vm = t.M - row0 - wr, vn = t.N - col0 - wc;
  bool ua[AB], ub[BB];
#pragma unroll
  for (int a = 0; a < AB; ++a) ua[a] = vm > 16 * a;
#pragma unroll
  for (int b = 0; b < BB; ++b) ub[b] = vn > 16 * b;
  M::V cr[AB][BB], ci[AB][BB];
#pragma unroll
  for (int a = 0; a < AB; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      cr[a][b] = M::V{0, 0, 0, 0};
      ci[a][b] = M::V{0, 0, 0, 0};
    }
  // this lane's output rows and columns through the maps, read now so that the epilogue does
  // not wait for them (-1: outside C)
  int orow[AB][4], ocol[BB];
#pragma unroll
  for (int b = 0; b < BB; ++b) {
    const int j = col0 + wc + 16 * b + (lane & 15);
    ocol[b] = j < t.N ? ((SCAT && t.cmap) ? t.cmap[j] : j) : -1;
  }
#pragma unroll
  for (int a = 0; a < AB; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = row0 + wr + 16 * a + M::row(lane, r);
      orow[a][r] = i < t.M ? ((SCAT && t.rmap) ? t.rmap[i] : i) : -1;
    }
  auto krange = [&](const GemmSeg& g, int& b, int& e) {
    b = t.kchunk > 0 ? kc * t.kchunk : 0;
    e = t.kchunk > 0 ? min(g.K, b + t.kchunk) : g.K;
  };
  auto next_seg = [&](int s, GemmSeg& g, int& b, int& e) {
    for (; s < t.nseg; ++s) {
      g = segs[t.seg_begin + s];
      krange(g, b, e);
      if (b < e) break;
    }
    return s;
  };
  // this lane's copies: A copy q of the wavefront is k = c / (TM / 64), rows 64 (c % (TM / 64))
  // + lane, with c = NLA wave + q; B copy q holds tile column j = 4 (NLA wave + q) + lane / 16
  // at swizzled k = (lane % 16) ^ (j % 16). A transposed (OPA 1, 2: rows of op(A) are columns
  // of the stored matrix, contiguous in k) is copied like B: [TM rows][16 k], swizzled.
  int arow[NLA], ak[NLA], bcol[NLA], bk[NLA];
#pragma unroll
  for (int q = 0; q < NLA; ++q) {
    const int c = NLA * wave + q;
    const int j = 4 * c + (lane >> 4);
    if (OPA == 0) {
      ak[q] = c / (TM / 64);
      arow[q] = min(row0 + 64 * (c % (TM / 64)) + lane, t.M - 1);
    } else {
      ak[q] = (lane & 15) ^ (j & 15);
      arow[q] = min(row0 + j, t.M - 1);
    }
    bcol[q] = min(col0 + j, t.N - 1);
    bk[q] = (lane & 15) ^ (j & 15);
  }
  auto issue = [&](int buf, const GemmSeg& g, int k0, int kend) {
    zd* la = lds + (size_t)buf * 32 * TM;
    zd* lb = la + 16 * TM;
#pragma unroll
    for (int q = 0; q < NLA; ++q) {
      const int c = NLA * wave + q;
      const zd* src = OPA == 0 ? g.A + arow[q] + (int64_t)min(k0 + ak[q], kend - 1) * g.lda
                               : g.A + min(k0 + ak[q], kend - 1) + (int64_t)arow[q] * g.lda;
      __builtin_amdgcn_global_load_lds(src, (void __attribute__((address_space(3)))*)(la + 64 * c), 16, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < NLA; ++q) {
      const int c = NLA * wave + q;
      const zd* src = g.B + min(k0 + bk[q], kend - 1) + (int64_t)bcol[q] * g.ldb;
      __builtin_amdgcn_global_load_lds(src, (void __attribute__((address_space(3)))*)(lb + 64 * c), 16, 0, 0);
    }
  };
  int nsteps = 0;
  for (int q = 0; q < t.nseg; ++q) {
    int b, e;
    krange(segs[t.seg_begin + q], b, e);
    if (b < e) nsteps += (e - b + BK - 1) / BK;
  }
  GemmSeg lg;
  int lk, le;
  int ls = next_seg(0, lg, lk, le);
  // per buffer: valid k count, and the row of A whose entry at k = 0 of the step carries the
  // shifted identity (A - E, E[ishift - 1 + k, k] = 1; -1 if none)
  int kval[2] = {0, 0}, kdiag[2] = {-1, -1};
  auto note = [&](int buf) {
    kval[buf] = le - lk;
    kdiag[buf] = lg.ishift > 0 ? lg.ishift - 1 + lk : -1;
  };
  if (nsteps > 0) {
    issue(0, lg, lk, le);
    note(0);
    lk += BK;
    if (lk >= le) ls = next_seg(ls + 1, lg, lk, le);
  }
  const int cl = lane & 15, kq = lane >> 4;
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's copies of step st have landed
    __syncthreads();                // everyone's have, and step st - 1 is no longer read
    if (st + 1 < nsteps) {
      issue(buf ^ 1, lg, lk, le);
      note(buf ^ 1);
      lk += BK;
      if (lk >= le) ls = next_seg(ls + 1, lg, lk, le);
    }
    const int kv = kval[buf], kd = kdiag[buf];
    const zd* As = lds + (size_t)buf * 32 * TM;
    const zd* Bs = As + 16 * TM;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int k = ks + kq;
      const bool kin = k < kv;
      zd av[AB], bv[BB];
#pragma unroll
      for (int a = 0; a < AB; ++a) {
        if (OPA == 0) {
          av[a] = As[k * TM + wr + 16 * a + cl];
          if (!SCAT && kd >= 0 && row0 + wr + 16 * a + cl == kd + k) av[a].re -= 1.0;
        } else {
          const int rr = wr + 16 * a + cl;
          av[a] = As[rr * 16 + (k ^ (rr & 15))];
          if (OPA == 2) av[a].im = -av[a].im;
        }
        if (!kin) av[a] = zd{0.0, 0.0};
      }
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        const int c = wc + 16 * b + cl;
        bv[b] = Bs[c * 16 + (k ^ (c & 15))];
      }
#pragma unroll
      for (int a = 0; a < AB; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b) {
          if (!(ua[a] && ub[b])) continue;
          cr[a][b] = M::mma(av[a].re, bv[b].re, cr[a][b]);
          cr[a][b] = M::mma(-av[a].im, bv[b].im, cr[a][b]);
          ci[a][b] = M::mma(av[a].re, bv[b].im, ci[a][b]);
          ci[a][b] = M::mma(av[a].im, bv[b].re, ci[a][b]);
        }
    }
  }
  const zd alpha{t.alpha_re, t.alpha_im};
  CT* Cb = static_cast<CT*>(t.C) + (int64_t)kc * t.part_stride;
#pragma unroll
  for (int b = 0; b < BB; ++b) {
    if (ocol[b] < 0) continue;
    // all old values of the column block first (in flight together: the entries are
    // distinct, which the compiler cannot see through the maps), then the stores
    zd old[AB][4];
    if (t.beta != 0.0) {
#pragma unroll
      for (int a = 0; a < AB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          old[a][r] = orow[a][r] >= 0 ? widen(Cb[orow[a][r] + (int64_t)ocol[b] * t.ldc]) : zd{0.0, 0.0};
    }
#pragma unroll
    for (int a = 0; a < AB; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (orow[a][r] < 0) continue;
        zd v = zmul(alpha, zd{(double)cr[a][b][r], (double)ci[a][b][r]});
        if (t.beta != 0.0) v = zadd(v, zscale(old[a][r], t.beta));
        Cb[orow[a][r] + (int64_t)ocol[b] * t.ldc] = narrow<CT>(v);
      }
  }
}

}  // namespace

// LDS of the direct-copy kernels: two buffers of A and B (16 K steps of TM complex each)
constexpr size_t kLdsGemmBytes64 = 2 * 32 * 64 * sizeof(zd);

int gemm_default_kernel(bool c32, bool mapped, int) {
  if (c32) return mapped ? GK_REG8 : GK_REG4;
  return GK_LDS;
}

void launch_gemm(int opA, const GemmTask* tasks, int ntasks, int64_t nunits, const GemmSeg* segs, bool c32,
                 hipStream_t st, bool mapped, const int32_t* utask, int kernel) {
  if (ntasks <= 0 || nunits <= 0) return;
  if (opA < 0 || opA > 2) throw Error(FMMLU_EINVAL, "GEMM op(A) must be 0, 1 or 2");
  if (mapped && opA != 0) throw Error(FMMLU_EINVAL, "mapped GEMM takes opA = N");
  if (c32 && opA != 0) throw Error(FMMLU_EINVAL, "float32 GEMM takes opA = N");
  const int k = kernel == GK_AUTO ? gemm_default_kernel(c32, mapped, opA) : kernel;
  if (k != GK_LDS && k != GK_REG8 && k != GK_REG4) throw Error(FMMLU_EINVAL, "unknown GEMM kernel");

  const dim3 g((unsigned)nunits), b4(256), b8(512);
#define FMMLU_GEMM_REG(OP, CT, SC)                                                                     \
  do {                                                                                                \
    if (k == GK_REG8)                                                                                 \
      hipLaunchKernelGGL((zgemm_mfma_kernel<OP, CT, SC, 8>), g, b8, 0, st, tasks, ntasks, segs, utask); \
    else                                                                                              \
      hipLaunchKernelGGL((zgemm_mfma_kernel<OP, CT, SC, 4>), g, b4, 0, st, tasks, ntasks, segs, utask); \
  } while (0)
  if (c32 && k == GK_LDS) {
    // float64 products rounded to float32 as they are stored
    if (mapped)
      hipLaunchKernelGGL((zgemm_lds_kernel<0, true, 64, zf>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
    else
      hipLaunchKernelGGL((zgemm_lds_kernel<0, false, 64, zf>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
  } else if (c32) {
    if (mapped)
      FMMLU_GEMM_REG(0, zf, true);
    else
      FMMLU_GEMM_REG(0, zf, false);
  } else if (k == GK_LDS) {
    if (mapped)
      hipLaunchKernelGGL((zgemm_lds_kernel<0, true, 64>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
    else if (opA == 0)
      hipLaunchKernelGGL((zgemm_lds_kernel<0, false, 64>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
    else if (opA == 1)
      hipLaunchKernelGGL((zgemm_lds_kernel<1, false, 64>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
    else
      hipLaunchKernelGGL((zgemm_lds_kernel<2, false, 64>), g, b8, kLdsGemmBytes64, st, tasks, ntasks, segs, utask);
  } else if (mapped) {
    FMMLU_GEMM_REG(0, zd, true);
  } else if (opA == 0) {
    FMMLU_GEMM_REG(0, zd, false);
  } else if (opA == 1) {
    FMMLU_GEMM_REG(1, zd, false);
  } else {
    FMMLU_GEMM_REG(2, zd, false);
  }
#undef FMMLU_GEMM_REG
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
