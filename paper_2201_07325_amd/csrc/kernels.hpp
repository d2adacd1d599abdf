// Task descriptors and launchers of the device kernels. Every kernel is batched over a
// list of independent tasks of uneven size; the host fills the task arrays, copies them
// to the device once per launch group, and a workgroup finds its task by binary search
// over the tasks' prefix sums of work units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace fmmlu {

// Quadrature corrections on the device (Section 5.3's locally corrected near field): the
// entry of a listed pair (i, j), i != j, is multiplied by 1 + a_ij (target-dependent weight
// w_ij = w_j (1 + a_ij)). CSR by row in tree positions, columns ascending, and the same
// pairs by column (for products with the conjugate transpose).
struct DevCorr {
  const int64_t* rptr = nullptr;  // n + 1
  const int32_t* rcol = nullptr;  // column of each entry
  const double* ra = nullptr;     // a_ij
  const int64_t* cptr = nullptr;  // n + 1, by column
  const int32_t* crow = nullptr;  // row of each entry
  const double* ca = nullptr;
};

// Geometry on the device, structure of arrays in tree order: x, y, z, nx, ny, nz, sqrt(w);
// corrections when the system has them (corr.rptr != nullptr).
struct DevGeom {
  const double* p;  // 7 * n doubles
  int64_t n;
  double k, eta;
  DevCorr corr;
  double kr_max = __builtin_inf();  // upper bound of k |x_i - x_j| over the points (inf: unknown)
};

// ---- tile assembly: out block = copy from old tiles where stored, else kernel entries ----
// Rows of the output are described by (slot, index) pairs: slot selects a source row group
// (a sub-owner) and index the row inside that group's source tile. Columns likewise. The
// source table holds, per (row slot, column slot), the source tile offset (-1: generate
// from the kernel) and its leading dimension.
struct AsmTask {
  int64_t out_off;      // destination offset (elements)
  int32_t nr, nc, ld;   // block size and destination leading dimension
  int32_t nsc;          // number of column slots (table row stride)
  int64_t rmap_off;     // offset into map arrays: rslot/ridx for rows
  int64_t cmap_off;     // ... cslot/cidx for columns
  int64_t rdof_off;     // offset into dof array: tree position of each output row
  int64_t cdof_off;     // ... of each output column
  int64_t tab_off;      // offset into the source table
  int64_t unit_begin;   // prefix sum of 64x64 work units
};
struct AsmSrc {
  int64_t off;  // source offset, -1 to generate
  int32_t ld;
  int32_t pad;
};

void launch_assemble(const DevGeom& g, const AsmTask* tasks, int ntasks, int64_t nunits,
                     const int32_t* slot, const int32_t* idx, const int64_t* dof,
                     const AsmSrc* table, const void* src_pool, bool src32, void* dst_pool, bool dst32,
                     hipStream_t st, const int32_t* utask = nullptr);

// ---- ID matrix [A_QB ; A_BQ^T ; proxy outgoing ; proxy incoming] (column-major) ----
struct QSeg {
  int64_t tile_qb;      // offset of tile (q, B): rows = act(q), cols = act(B); -1: generate
  int64_t tile_bq;      // offset of tile (B, q): rows = act(B), cols = act(q)
  const int32_t* live;  // live rows of q (positions in act(q))
  const int64_t* gdof;  // generated segments: tree positions of act(q) (a spill-over owner
                        // beyond the stored tiles: its entries are corrected kernel values)
  int32_t ld;           // |act(q)|, leading dimension of tile (q, B)
  int32_t row0;         // first row of this segment inside the A_QB block
};
struct IdTask {
  zd* M;             // output matrix
  int32_t rows, m;   // M is rows x m, ld = rows
  int32_t nq;        // sum of Q counts
  int32_t ngamma;    // proxy points (0: no proxy rows)
  int32_t nseg;      // number of Q segments
  int32_t pad;
  int64_t seg_off;   // offset into QSeg array
  int64_t dof_off;   // tree positions of B's active DOFs (m)
  double cx, cy, cz, radius, wgamma;  // proxy sphere centre, radius, row weight
  int64_t unit_begin;
};
void launch_build_idmatrix(const DevGeom& g, const IdTask* tasks, int ntasks, int64_t nunits,
                           const QSeg* segs, const int64_t* dof, const void* pool, bool pool32, hipStream_t st);

// ---- batched complex GEMM with segments and scatter maps ----
// C[rmap[i], cmap[j]] = beta * C[...] + alpha * sum_s opA(A_s)[i, :] * B_s[:, j]
// opA: 0 = N (A is M x K, lda), 1 = T (A stored K x M), 2 = C (conjugate transpose).
constexpr int kGemmTile = 64;  // C block per workgroup (kGemmTile x kGemmTile)
struct GemmSeg {
  const zd* A;
  const zd* B;
  int32_t lda, ldb, K;
  int32_t ishift;  // opA N only: > 0 reads A - E with E[ishift - 1 + k, k] = 1 (shifted identity)
};
struct GemmTask {
  void* C;  // complex float64, or float32 for launches with c32
  const int32_t* rmap;  // may be null (identity)
  const int32_t* cmap;  // may be null (identity)
  const int32_t* skip;  // may be null; the task is skipped when *skip != 0 at launch time
  int32_t M, N, ldc;
  int32_t seg_begin, nseg;
  int32_t kchunk;                   // > 0: split K into chunks; chunk c writes C + c*part_stride
  int32_t lower;                    // M == N: only the output tiles on or below the diagonal
  int32_t pad;
  double alpha_re, alpha_im, beta;  // beta real
  int64_t part_stride;
  int64_t unit_begin;              // prefix sum of kGemmTile^2 output blocks (times K chunks)
};
// output blocks (tile x tile) of one K chunk of a task: all, or the T (T + 1) / 2 on or
// below the diagonal
__host__ __device__ inline int64_t gemm_task_tiles_t(int M, int N, int lower, int tile) {
  const int64_t tm = (M + tile - 1) / tile, tn = (N + tile - 1) / tile;
  return lower ? tm * (tm + 1) / 2 : tm * tn;
}
__host__ __device__ inline int64_t gemm_task_tiles(int M, int N, int lower) {
  return gemm_task_tiles_t(M, N, lower, kGemmTile);
}
// Kernels of the batched GEMM (all 64 x 64 output blocks): operands copied straight into
// double-buffered LDS by eight wavefronts (float64 products; a float32 C gets them rounded as
// stored), or staged through registers by eight or four wavefronts (float32 C: float32
// products). GK_AUTO: the library's default for the use, gemm_default_kernel.
enum GemmKernel { GK_AUTO = -1, GK_LDS = 0, GK_REG8 = 1, GK_REG4 = 2 };
int gemm_default_kernel(bool c32, bool mapped, int opA);
// mapped: tasks may carry rmap / cmap (a separate kernel instance); otherwise they are ignored.
// utask (optional, nunits entries): the task of each output block, in place of a search of
// the tasks' unit_begin prefix sums. kernel: a GemmKernel.
void launch_gemm(int opA, const GemmTask* tasks, int ntasks, int64_t nunits, const GemmSeg* segs, bool c32,
                 hipStream_t st, bool mapped = false, const int32_t* utask = nullptr, int kernel = GK_AUTO);


// ---- Householder panel factorization (unpivoted QR) ----
struct QrTask {
  zd* A;          // matrix, column-major, lda
  zd* V;          // output: explicit reflectors (rows - j0) x nb, ld = rows - j0
  zd* Tw;         // output: nb x nb triangular factor of the compact WY form
  int32_t rows, lda, j0, nb;
};
void launch_qr_panel(const QrTask* tasks, int ntasks, hipStream_t st);
constexpr int kQrBlock = 16;  // panel width of the blocked Householder QR
// W2 = Tw^H * sum_k part_k  (part_k: nb x ncols, ld nb, stride part_stride)
struct RedTwTask {
  const zd* part;
  const zd* Tw;
  zd* W2;
  int32_t nb, ncols, nsplit, pad;
  int64_t part_stride;
};
void launch_reduce_tw(const RedTwTask* tasks, int ntasks, int nmax, hipStream_t st);

// ---- greedy CPQR on an m x m matrix (in place) + T = R11^{-1} R12 ----
struct CpqrTask {
  zd* R;           // m x m, ld = lda (in place)
  int32_t* perm;   // output m
  int32_t* rank;   // output (device scalar)
  zd* T;           // output s x (m - s), ld = m (room for s <= m)
  zd* W;           // scratch, m * m / 4 + m entries
  int32_t m, lda;
};
void launch_cpqr(const CpqrTask* tasks, int ntasks, int mmax, double eps, hipStream_t st);

// ---- gathers of the cross of B ----
// With perm the ID pivot order (skeletons S = perm[0:s], redundant R = perm[s:m]):
//   Ccol = A[(R, S, N), (S, R)]   ((m + nN) x m, ld m + nN)
//   Crow = A[(S, R), (R, S, N)]   (m x (m + nN), ld m)
// so that after the E/F transforms X_RR, X_{(S u N) R} and X_{R (S u N)} are contiguous.
struct NSeg {
  int64_t tile_nb;      // tile (o, B): rows act(o), ld = ld
  int64_t tile_bn;      // tile (B, o): rows act(B), ld = m
  const int32_t* live;  // live rows of o
  int32_t ld, off;      // |act(o)| and position of its first live DOF in the N list
};
struct CrossTask {
  zd* Ccol;  // (m + nN) x m, ld = m + nN
  zd* Crow;  // m x (m + nN), ld = m
  int64_t tile_bb;   // tile (B, B), ld = m
  const int32_t* perm;
  int32_t m, nN, nseg, s;
  int64_t seg_off;
  int64_t unit_begin;
};
void launch_gather_cross(const CrossTask* tasks, int ntasks, int64_t nunits, const NSeg* segs,
                         const void* pool, bool pool32, hipStream_t st);

// ---- sum of split-K partials: out[e] = sum_k part[k*stride + e], e < count ----
// herm = m > 0: out is m x m (count = m m) and only the lower triangle's partials exist; the
// sum goes to the lower triangle and its conjugate to the upper (a full Hermitian matrix)
struct SumTask {
  const zd* part;
  zd* out;
  int64_t count, stride;
  int32_t nsplit, herm;
  int64_t unit_begin;  // units of 256 elements
};
void launch_sum_parts(const SumTask* tasks, int ntasks, int64_t nunits, hipStream_t st);

// ---- greedy CPQR through the Gram matrix: pivoted Cholesky of G = M^H M (m x m) ----
// Left-looking: row k of R from column p_k of G and the previous rows; the diagonal of the
// Schur complement (the squared norms of the remaining columns after projection) is updated
// exactly. Outputs as CpqrTask: perm, rank, T = R11^{-1} R12 (ld m).
struct PcholTask {
  zd* G;           // m x m, ld m, Hermitian, both triangles (the blocked form overwrites it)
  zd* Rt;          // m x m scratch: rows of R by original column, Rt[l * m + c]
  zd* Rp;          // m x m scratch: R in pivoted column order, ld m
  int32_t* perm;
  int32_t* rank;
  zd* T;
  int32_t m, pad;
  // blocked form only: the block's rows of R (kPcholNb x m, column-major), and the state
  // kept between block launches (dg and r00: m + 1 doubles; pos, pv, then k, done: 2m + 2)
  zd* Rb;
  double* dgs;
  int32_t* ist;
};
// Blocked greedy pivoted Cholesky (matrices of m <= kPcholThreadsB columns): launch block
// b = 0, 1, ... takes pivots kPcholNb b .. kPcholNb (b + 1) - 1 left-looking within the block
// (rows of the block in registers, one column per thread) against G, then the caller
// downdates G -= Rb^H Rb (both triangles) before the next block; pchol_finish writes rank,
// perm and R in pivoted order. Equal to launch_pchol's result in exact arithmetic.
constexpr int kPcholNb = 16;
constexpr int kPcholThreadsB = 1024;
constexpr int kPcholBlockedMin = 128;  // widest block of a phase from which the blocked form is used
void launch_pchol_block(const PcholTask* tasks, int ntasks, int k0, double eps, hipStream_t st, int mmax);
void launch_pchol_finish(const PcholTask* tasks, int ntasks, int mmax, hipStream_t st);
void launch_pchol(const PcholTask* tasks, int ntasks, int mmax, double eps, hipStream_t st);
// after launch_pchol or launch_pchol_finish: T = R11^{-1} R12 by back substitution (rank and
// perm are final before it, so their read-back can be queued ahead of it)
void launch_pchol_t(const PcholTask* tasks, int ntasks, int mmax, hipStream_t st);

// ---- Gauss-Jordan inversion with partial pivoting, blocked ----
struct GjTask {
  zd* A;      // n x n, ld = lda
  int32_t* piv;
  int32_t n, lda;
  int32_t* info;  // set to 1 + column on a zero pivot; -1 if a panel barrier timed out
  // panel: one row per thread, kGjPanelRows rows per workgroup, wpt workgroups per matrix.
  // With wpt > 1 the workgroups exchange pivot candidates through slots (2 x gj_slot_len)
  // and meet at a barrier counter that must be zero before the first panel.
  zd* slots;
  int32_t* counter;
  int32_t wpt, pad;
};
constexpr int kGjBlock = 16;  // Gauss-Jordan panel width
constexpr int kGjPanelRows = 256;
__host__ __device__ inline int gj_wpt(int n) { return (n + kGjPanelRows - 1) / kGjPanelRows; }
// entries of one slot buffer: per workgroup a candidate (|pivot|^2, row) and its row values,
// then the values of the row at the pivot position
__host__ __device__ inline int64_t gj_slot_len(int wpt) { return (int64_t)wpt * (kGjBlock + 1) + kGjBlock; }
// grid ntasks x wmax; cooperative when wmax > 1 (then ntasks * wmax <= gj_panel_capacity())
void launch_gj_panel(const GjTask* tasks, int ntasks, int j0, int wmax, hipStream_t st);
int gj_panel_capacity();
// Whole inversion of matrices of n <= kGjCoopMax rows in one cooperative launch: nwg
// workgroups per matrix starting at grid index unit_begin; out = A^{-1} (n x n, ld n);
// counter: gj_coop_sync_words zeroed words. Panels of gj_coop_panel(nmax) columns, nmax the
// largest n of the launch.
constexpr int kGjCoopMax = 512;
struct GjCoopTask {
  zd* A;
  zd* out;
  int32_t* piv;
  int32_t* info;
  int32_t* counter;  // gj_coop_sync_words(n) zeroed words
  int32_t n, lda, nwg, pad;
  int64_t unit_begin;
};
inline int gj_coop_panel(int) { return 16; }
// synchronisation words of one matrix: panel-ready flags, panel-read counts, final count
inline int gj_coop_sync_words(int n, int nb) { return 2 * ((n + nb - 1) / nb) + 1; }
void launch_gj_coop(const GjCoopTask* tasks, int ntasks, int64_t nwg_total, int nmax, hipStream_t st);
// workgroups of gj_coop that can be resident at once; compute units of the device
int gj_coop_capacity(int nmax);
int gj_coop_cus();

// Stepped Gauss-Jordan inversion of one matrix of kGjCoopMax < n <= kGjStepMax rows with
// implicit pivoting, one launch per panel of kGjStepNb columns (the launch boundary is the
// only synchronisation between workgroups). Launch j: workgroup 0 applies panel j to the
// columns of panel j + 1 and factors that panel; the other workgroups apply panel j to every
// other column. piv (n): pivot row of each column; rowcol (n, all -1 before the first
// launch): the column each row pivots. After the last step out[i, c] = M[piv[i], rowcol[c]]
// (launch_gj_step_gather). info as for the other inversions.
constexpr int kGjStepMax = 2048;
constexpr int kGjStepNb = 8;
constexpr int kGjStepThreads = 512;
struct GjStepArgs {
  zd* A;
  int32_t* piv;
  int32_t* rowcol;
  int32_t* info;
  int32_t n, lda;
};
void launch_gj_step(const GjStepArgs& a, int j, hipStream_t st);  // j = -1 .. npan - 1
void launch_gj_step_gather(const GjStepArgs& a, zd* out, hipStream_t st);
// marks a factorization in progress for the lifetime of the object (cooperative launches are
// serialised while more than one is active)
struct ActiveFactorization {
  ActiveFactorization();
  ~ActiveFactorization();
  static int count();  // factorizations in progress in the process
};
void launch_gj_swaps(const GjTask* tasks, int ntasks, int j0, int nmax, hipStream_t st);
// W (nb x n) = A[J, :] with J = [j0, j0+nb)
void launch_gj_copyrow(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W,
                       hipStream_t st);
// row exchanges of the panel on columns outside J, then W (nb x n) = A[J, :]
void launch_gj_swapcopy(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W, hipStream_t st);
// A[J, c] -= W[:, c] for c outside J
void launch_gj_fixrow(const GjTask* tasks, int ntasks, int j0, int nmax, zd* const* W,
                      hipStream_t st);
// undo the column permutation: Out = A * P (gather columns)
void launch_gj_unpermute(const GjTask* tasks, int ntasks, int nmax, zd* const* out,
                         int32_t* const* work, hipStream_t st);

// ---- R factor extraction: R = triu(M[0:min(rows,m), 0:m]) padded to m x m ----
struct ExtractTask {
  const zd* M;
  zd* R;
  int32_t rows, m;
};
void launch_extract_r(const ExtractTask* tasks, int ntasks, int mmax, hipStream_t st);

// ---- copy a sub-block (column-major) ----
struct CopyTask {
  const zd* src;
  void* dst;  // complex float64, or float32 with dst32
  int32_t rows, cols, lds, ldd;
  int64_t unit_begin;
  int32_t transpose;  // 0: dst[i + j*ldd] = src[i + j*lds]; 1: dst[j + i*ldd] = src[i + j*lds]
  int32_t pad;
};
// copies and transposes of rows x cols sources; units of 64 x 64
void launch_copy(const CopyTask* tasks, int ntasks, int64_t nunits, bool dst32, hipStream_t st);

// ---- solve sweeps ----
struct SolveBox {
  const int32_t* R;   // tree positions, r
  const int32_t* S;   // s
  const int32_t* SN;  // s + nN (S first)
  // factors, complex float64 or float32 (the factorization's storage precision)
  const void* T;      // s x r, ld = s
  const void* Xi;     // r x r inverse pivot block
  const void* Lp;     // L = X_{(S u N) R} X_RR^{-1}: (s+nN) x r, ld = s+nN
  const void* UpT;    // U^T with U = X_RR^{-1} X_{R (S u N)}: (s+nN) x r, ld = s+nN
  int32_t r, s, nsn;
  int32_t nks;        // chunks of kSolveK over s (forward x_R partials)
  int32_t nchunk;     // chunks of kSolveK over s + nN (backward x_R partials)
  int32_t pad;
  int64_t y_off;      // this box's outputs in the forward scatter buffer
  int64_t p_off;      // backward x_R partials (nchunk x r)
  int64_t xrp_off;    // forward x_R partials (nks x r)
  int64_t dx_off;     // this box's x_R in the buffer of all boxes (sum of r)
};
// Work item of a sweep kernel: rows or columns [k0, k0 + kn) of box `box`; `chunk` is the
// k-chunk and `grp` the group of kSolveOut outputs (column GEMVs).
struct SweepTask {
  int32_t box, k0, kn, chunk, grp, pad;
};
constexpr int kSolveRows = 64;   // rows per row-GEMV work item (one row per lane)
constexpr int kSolveK = 256;     // k-chunk of column GEMVs (over s or s + nN) and of staged x_R
constexpr int kSolveOut = 64;    // outputs per column-GEMV work item
// sweeps: a step whose phase has fewer items of 64 than this (two per compute unit) runs in
// items of 16 outputs or rows instead
constexpr int kSolveFineBelow = 512;

// Vectors inside the sweeps are interleaved (entry i of right-hand side c at [i nr + c]):
// nr = 1 for the single-vector kernels below, nr = kSolveBlock for the blocked ones (matrix
// cores, launch_blk_*); the permutations, scatter and top-block gather and sum take either.
constexpr int kSolveBlock = 32;
constexpr int kApplyK = 64;  // k-chunk of the staged vector block in the blocked sweeps (32 KiB)
// Single-vector sweep steps. Column products take output groups of gsz (64, or 16 on phases
// with few work items: task grp g covers outputs [g gsz, (g + 1) gsz)); row products take
// items of `rows` (64 or 16) rows.
// forward: partials of op(T)^T x_S (T^T, adjoint T^H) per (box, s-chunk, output group)
void launch_solve_xr_part(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pxr,
                          int adjoint, bool f32, hipStream_t st, int nr = 1);
// forward, per (box, item of rows of S u N): x_R = x[R] - sum of the partials (kept in XRg by
// the item of the first rows), then y = op(P) x_R (Lp, adjoint conj(Up^T)) for those rows
// (direct: no two boxes of the phase share a row of S u N; the rows are subtracted from x
// here and the phase needs no scatter)
void launch_solve_y(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, zd* x, const zd* Pxr,
                    zd* XRg, zd* y, int adjoint, int direct, bool f32, hipStream_t st, int nr = 1);
// x[dst[d]] -= sum of y[src[q]] over ptr[d] <= q < ptr[d+1] (deterministic scatter)
void launch_scatter_sub(const int32_t* dst, const int64_t* ptr, const int64_t* src, int64_t nd,
                        const zd* y, zd* x, hipStream_t st, int nr = 1);
// diagonal: XRd = Xi XRg (adjoint Xi^H XRg) for every box, items (box, 64 outputs) with box
// indexing the table of all boxes (rmax 16 bytes of LDS <= 64 KiB)
void launch_solve_diag(const SolveBox* boxes, const SweepTask* tasks, int nt, int rmax, const zd* XRg, zd* XRd,
                       int adjoint, bool f32, hipStream_t st, int nr = 1);
// backward: partials of op(Q)^T x_SN (Up, adjoint Lp^H) per (box, column chunk, output group)
void launch_solve_bpart(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pbuf,
                        int adjoint, bool f32, hipStream_t st, int nr = 1);
// backward, per (box, item of rows of S): x_R = XRd - sum of the partials (written to x[R] by
// the item of the first rows), then x_S -= op(T) x_R (T, adjoint conj(T)) for those rows
void launch_solve_bt(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, const zd* XRd,
                     const zd* Pbuf, zd* x, int adjoint, bool f32, hipStream_t st, int nr = 1);
// The same steps for blocks of kSolveBlock right-hand sides on the matrix cores (the same work
// items, with output groups or row items of 16 or 64 chosen per phase, and items of 16 rows of
// S for launch_blk_bt; the pivot blocks take one item per (box, 64 outputs) with box indexing
// the table of all boxes; the top block's partials over chunks of 256 go to
// launch_solve_top_fin).
void launch_blk_xr_part(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pxr,
                        int adjoint, bool f32, hipStream_t st);
void launch_blk_y(const SolveBox* boxes, const SweepTask* tasks, int nt, int rows, zd* x, const zd* Pxr,
                  zd* XRg, zd* y, int adjoint, int direct, bool f32, hipStream_t st);
void launch_blk_diag(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XRg, zd* XRd, int adjoint,
                     bool f32, hipStream_t st);
void launch_blk_bpart(const SolveBox* boxes, const SweepTask* tasks, int nt, int gsz, const zd* x, zd* Pb,
                      int adjoint, bool f32, hipStream_t st);
// backward x_R = XRd - sum of the partials per (box, 64 entries of R), stored back to XRd and
// to x[R]; launch_blk_bt with presummed = 1 then stages XRd alone
void launch_blk_xr_sub(const SolveBox* boxes, const SweepTask* tasks, int nt, zd* XRd, const zd* Pb, zd* x,
                       hipStream_t st);
void launch_blk_bt(const SolveBox* boxes, const SweepTask* tasks, int nt, const zd* XRd, const zd* Pb, zd* x,
                   int adjoint, int presummed, bool f32, hipStream_t st);
void launch_blk_top_part(const zd* Ainv, int n0, const zd* tmp, zd* part, int adjoint, hipStream_t st);
// top block: x_t = Ainv x_t (adjoint Ainv^H); tmp holds n0 (1 + nblk) nr entries, nblk =
// ceil(n0 / 256). Blocked: gather, launch_blk_top_part on (tmp, tmp + n0 nr), then the sum
void launch_solve_top(const zd* Ainv, int n0, const int32_t* top, zd* x, zd* tmp, int adjoint,
                      hipStream_t st, int nr = 1);
void launch_solve_top_gather(int n0, const int32_t* top, const zd* x, zd* tmp, hipStream_t st, int nr);
void launch_solve_top_fin(int n0, const int32_t* top, const zd* part, zd* x, hipStream_t st, int nr);
// permute between the caller's column-major vectors (ld, m <= nr active columns) and the
// interleaved tree-order block: gather dst[i nr + c] = src[map[i] + c ld] (zero for c >= m),
// or scatter dst[map[i] + c ld] = src[i nr + c] for c < m
void launch_permute(const zd* src, zd* dst, const int64_t* map, int64_t n, int gather,
                    hipStream_t st, int nr = 1, int64_t ld = 0, int m = 1);

// ---- stand-alone block of A~ (rows, cols: tree positions) ----
void launch_block(const DevGeom& g, const int64_t* rows, int64_t nr, const int64_t* cols,
                  int64_t nc, zd* out, hipStream_t st);

// ---- vector kernels of the refinement ----
constexpr int kDotBlocks = 512;  // fixed partition of inner products (deterministic)
void launch_dotc_partial(const zd* x, const zd* y, int64_t n, zd* part, hipStream_t st);
void launch_axpy(zd a, const zd* x, zd* y, int64_t n, hipStream_t st);
void launch_scal_copy(zd a, const zd* x, zd* y, int64_t n, hipStream_t st);
void launch_sub(const zd* a, const zd* b, zd* out, int64_t n, hipStream_t st);

// ---- far-field pattern operator ----
// op 0: out(ndir) = C in(n); 1: out(n) = C^H in(ndir); 2: dC/dk; 3: dC/deta (as op 0).
// part holds ndir * farfield_chunks(n) entries (ops 0, 2, 3).
constexpr int64_t kFarChunk = 4096;
int farfield_chunks(int64_t n);
void launch_farfield(const DevGeom& g, int op, const double* dirs, int64_t ndir, const int64_t* order,
                     const zd* in, zd* out, zd* part, hipStream_t st);

// ---- exact matvec on the fly ----
// part: part_entries scratch entries for the partial sums of the source slices, at least
// matvec_slices(n, part_entries) * n. The slice count (at most kMatvecMaxSlices and
// max_entries / n) is the one whose workgroups fill the current device's resident slots best,
// fixed per device and n.
constexpr int kMatvecMaxSlices = 16;
int matvec_slices(int64_t n, int64_t max_entries = INT64_MAX);
void launch_matvec(const DevGeom& g, int op, const zd* x, zd* y, zd* part, int64_t part_entries,
                   hipStream_t st);

// ---- allocation-free exact matvec ----
// One file-scope device array per GPU (kNoallocScratchBytes) holds the permuted input, the
// tree-order result and the slice partials: (2 + matvec_slices(n, matvec_noalloc_part_entries(n)))
// * n entries.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
int64_t matvec_noalloc_part_entries(int64_t n);  // room left for the partials after 2 n entries
int64_t matvec_noalloc_entries(int64_t n);
// device address of the current device's array (hipGetSymbolAddress on first use per device)
zd* noalloc_scratch();

}  // namespace fmmlu
