/*
 * fmmlu.h -- C ABI of the MI355X (gfx950) FMM-LU library.
 *
 * FMM-LU (Sushnikova, Greengard, O'Neil, Rachh) factors the dense Nystrom matrix of the
 * 3-D Helmholtz combined-field integral equation by recursive strong skeletonization over
 * a level-restricted adaptive octree (Sections 4.1-4.4), with far fields compressed
 * against proxy spheres (Sections 5.1-5.2). The system solved is the square-root-weighted
 * one of Section 3, eq. (disc3), with plain smooth weights w_j and alpha = 1/2:
 *
 *     A~_ii = 1/2,   A~_ij = sqrt(w_i) K(x_i, x_j) sqrt(w_j)  (i != j),
 *     K(x, y) = n(y) . grad_y G(x, y) - i eta G(x, y),   G = e^{ik|x-y|} / (4 pi |x-y|)
 *
 * (eq. comb_ref with the single-layer coupling k generalised to eta), acting on
 * sigma~ = sqrt(w) sigma with right-hand side b~ = sqrt(w) f.
 *
 * Conventions for every entry point:
 *   - Return value is an fmmlu_status; 0 means success. No function throws, aborts or
 *     exits across this boundary. On failure fmmlu_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Geometry (points, normals, weights) is HOST memory, structure-of-arrays float64:
 *     xyz[0..n) = x, xyz[n..2n) = y, xyz[2n..3n) = z. The library copies what it keeps;
 *     the caller keeps ownership.
 *   - Vectors passed to solve / matvec are DEVICE memory, complex128 interleaved
 *     (re, im), column-major n x nrhs, in the caller's original point order. They are
 *     read and written on the caller's HIP stream (hip_stream == NULL means the null
 *     stream); calls return once the work is enqueued unless stated otherwise.
 *   - Handles are opaque and owned by the caller; destroy functions accept NULL.
 *   - A GPU runtime error is reported as FMMLU_EHIP with the HIP error string.
 */
#ifndef FMMLU_H
#define FMMLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMMLU_OK = 0,
  FMMLU_EINVAL = -1,     /* invalid argument: sizes, NaN/Inf, non-positive weight, duplicate point, ... */
  FMMLU_ENOMEM = -2,     /* device or host allocation failed, or the configured memory cap was exceeded */
  FMMLU_EHIP = -3,       /* HIP runtime error */
  FMMLU_ESINGULAR = -4,  /* a pivot block X_RR or the top block is numerically singular */
  FMMLU_ENOCONV = -5,    /* iterative refinement did not reach the tolerance */
  FMMLU_ESTATE = -6      /* handle in the wrong state (e.g. NULL factor) */
} fmmlu_status;

typedef enum {
  FMMLU_FP64 = 0,  /* complex float64 tiles, factors and solves */
  FMMLU_FP32 = 1   /* complex float32 tiles and factors; ID and pivot blocks in float64 */
} fmmlu_precision;

typedef struct fmmlu_tree_s* fmmlu_tree_h;
typedef struct fmmlu_factor_s* fmmlu_factor_h;
typedef struct fmmlu_batch_s* fmmlu_batch_h;

/* Options of fmmlu_factor. Fill with fmmlu_default_opts() first. */
typedef struct {
  double eps;                 /* ID tolerance, relative (Section 4.1 Definition); in (0, 0.1] */
  double proxy_radius;        /* proxy sphere radius in units of the box side (Section 4.4: 2.5) */
  int32_t proxy_min_points;   /* floor on proxy points per sphere (64) */
  int32_t precision;          /* fmmlu_precision */
  int64_t device_mem_cap;     /* bytes of device memory the factorization may hold (all of it:
                                 factors, tile pools, scratch, upload buffers); 0 = no cap.
                                 Exceeding it returns FMMLU_ENOMEM */
  int32_t verbose;            /* 0 silent, 1 per-level summary on stderr */
  int32_t profile;            /* 1: time each kernel class with HIP events (fmmlu_factor_profile);
                                 2: the Schur-update class (6) only, fewer event records */
  int32_t id_route;           /* greedy CPQR route: 0 auto (Gram matrix when eps >= 1e-7, else
                                 Householder), 1 Gram matrix + pivoted Cholesky, 2 Householder QR */
  int32_t test_zero_pivot_block; /* failure-path testing only: -1 (default) off; r >= 0 zeroes the
                                 pivot block X_RR of the r-th eliminated box before its inversion,
                                 so that the factorization returns FMMLU_ESINGULAR */
  /* Device memory. With alloc == NULL the library allocates with hipMalloc and keeps released
   * blocks in a process-wide cache for later factorizations (fmmlu_trim_caches frees it).
   * With alloc set, EVERY device block a factorization holds (geometry, factors, tile pools,
   * planning scratch, upload buffers, solve and refinement workspace) comes from
   * alloc(bytes, hip_stream, alloc_ctx) and goes back through free(ptr, hip_stream, alloc_ctx),
   * nothing is cached by the library, and a NULL return is reported as FMMLU_ENOMEM. A block is
   * handed to free only after the device has finished the work that used it, or with that
   * work ordered before anything later queued on the given stream (the factorization's stream,
   * or the null stream once fmmlu_factor has returned). Both functions must be thread-safe when
   * fmmlu_factor_batch uses them from several threads. */
  void* (*alloc)(size_t bytes, void* hip_stream, void* ctx);
  void (*free)(void* ptr, void* hip_stream, void* ctx);
  void* alloc_ctx;
  /* Locally corrected quadrature (Section 5.3), optional (all NULL: none): the weight of
   * source j at target i becomes w_j (1 + a_ij) for the listed pairs, i.e. the entry
   * A~_ij = sqrt(w_i) K(x_i, x_j) sqrt(w_j) is multiplied by 1 + a_ij. HOST arrays in the
   * original point order, CSR by target: for i < n the pairs (i, corr_col[e]) with factor
   * corr_a[e], e in [corr_row_ptr[i], corr_row_ptr[i + 1]); corr_row_ptr[0] = 0. Pairs with
   * j == i are ignored (the diagonal is 1/2); a pair listed twice is EINVAL. The library
   * copies the table. An owner box that a listed pair links to box B while lying in B's far
   * region P joins B's Q region for B's interpolative decomposition (its entries are not
   * kernel values, so the proxy surface cannot stand for them). fmmlu_factor only. */
  const int64_t* corr_row_ptr;
  const int64_t* corr_col;
  const double* corr_a;
  int32_t gemm_autotune;      /* 1 (default): before the first factorization on a device, time
                                 every kernel of the batched GEMM per use and K bucket on a
                                 synthetic batch and use the fastest (fmmlu_gemm_tuning); 0: the
                                 default kernels; 2, 3, 4 (testing): one kernel for every GEMM
                                 (direct-to-LDS where it applies, register-staged with eight or
                                 four wavefronts) */
  int32_t pchol_blocks;       /* 0 (default): the blocked pivoted Cholesky (Gram route, wide
                                 boxes) launches blocks of pivots up to a bound from the ranks
                                 seen so far, and the remaining blocks only when a box's pivoting
                                 has not stopped by then (found at the rank read-back); k > 0
                                 (testing): at most k blocks before the first read-back. The
                                 result is the same either way. */
  int32_t reserved[2];
} fmmlu_opts;

/* Per-factorization statistics. */
typedef struct {
  int64_t n;                  /* unknowns */
  int64_t n0;                 /* size of the top block B_t (Section 4.2) */
  int32_t nlevels;            /* octree levels, root = 0 */
  int32_t nboxes_factored;    /* boxes whose redundant DOFs were eliminated */
  int64_t factor_bytes;       /* device bytes held by the factors */
  int64_t peak_bytes;         /* peak device bytes held during the factorization: factors, tile
                                 pools, planning scratch and upload buffers together */
  int32_t max_rank;           /* largest skeleton size |S| */
  int32_t max_block;          /* largest active DOF count m of a box */
  double t_tree, t_factor;    /* seconds (host wall clock, device synchronised) */
  double flops_id, flops_elim, flops_schur, flops_top;  /* algorithmic flop counts */
  double bytes_tiles;         /* bytes of pair tiles generated or merged */
  int32_t precision;
  int32_t nspill;             /* Q-region additions for quadrature corrections reaching a box's
                                 far field (Section 5.3 spill-over), summed over boxes */
  int32_t reserved[6];
} fmmlu_info;

/* Fill *opts with defaults: eps 1e-6, proxy_radius 2.5, proxy_min_points 64, FP64. */
fmmlu_status fmmlu_default_opts(fmmlu_opts* opts);

/*
 * Build the level-restricted adaptive octree (Section 4, opening): root cube centred on
 * the points' bounding box with side (largest extent)*(1 + 1e-12); a box is split into
 * eight while it holds more than leaf_size points; leaves that share a boundary point
 * are then brought to within one level of each other by splitting the coarser one.
 * xyz: host, 3*n doubles (SoA). n >= 1, leaf_size >= 1. Points must be finite and
 * pairwise distinct (FMMLU_EINVAL otherwise). Host-only work.
 */
fmmlu_status fmmlu_build_tree(const double* xyz, int64_t n, int32_t leaf_size, fmmlu_tree_h* out);

/* Tree description for inspection: number of boxes, levels and leaves. Any output
 * pointer may be NULL. */
fmmlu_status fmmlu_tree_info(fmmlu_tree_h t, int64_t* nboxes, int32_t* nlevels, int64_t* nleaves);

/* Export the boxes: for box b, level[b], coord[3b..3b+2] (integer coordinates at its level),
 * npts[b] and is_leaf[b]; and the tree order of the points: order[i] = original index of
 * the i-th point in tree order (leaves by the Morton key of their lower corner, then by
 * original index). Host arrays sized by fmmlu_tree_info. Any pointer may be NULL. */
fmmlu_status fmmlu_tree_export(fmmlu_tree_h t, int32_t* level, int32_t* coord, int32_t* npts,
                               int8_t* is_leaf, int64_t* order);

void fmmlu_tree_destroy(fmmlu_tree_h t);

/*
 * Factor A~ by recursive strong skeletonization (Sections 4.1-4.4, 5.1-5.3 without
 * quadrature corrections) on the GPU of the calling thread's current HIP device.
 * The tree must have been built from the same points. normals: host 3*n unit vectors
 * (outward), weights: host n positive doubles. k >= 0 (k = 0 is the Laplace limit),
 * eta any finite real. The factor keeps its own device copy of the geometry and does
 * not reference the tree afterwards. Synchronises hip_stream before returning.
 * Errors: EINVAL (bad sizes/values), ENOMEM, EHIP, ESINGULAR.
 */
fmmlu_status fmmlu_factor(fmmlu_tree_h t, const double* xyz, const double* normals,
                          const double* weights, double k, double eta, const fmmlu_opts* opts,
                          void* hip_stream, fmmlu_factor_h* out);

/*
 * x = A_f^{-1} b with the factored inverse of Section 4.2:
 * A^{-1} ~ (W_1^{-1} ... W_M^{-1}) P_t D^{-1} P_t^T (V_M^{-1} ... V_1^{-1}).
 * b, x: device complex128, n x nrhs column-major (may alias: in-place is allowed).
 * nrhs > 1 is applied in blocks of 32 columns (a ragged last block padded with zeros), each
 * factor entry read once per block, on the matrix cores; a single column goes through the
 * single-vector sweeps. The two agree to rounding (different summation order); each is
 * deterministic run to run.
 */
fmmlu_status fmmlu_solve(fmmlu_factor_h f, const void* b, void* x, int64_t nrhs, void* hip_stream);

/*
 * Solve launch mode. By default (enable = 1) the first solve in each direction captures its
 * sweeps (kernels only) into a HIP graph on a private stream, and every solve then copies b
 * into the graph's input, replays the graph on hip_stream and copies the result out: the
 * same kernels in the same order, with one launch instead of a few hundred. enable = 0
 * launches the kernels one by one on hip_stream (needed by callers that capture solves into
 * graphs of their own). If capture is not possible the library falls back to enable = 0.
 * Concurrent solves on one factor must be serialised by the caller (they share workspace).
 */
fmmlu_status fmmlu_set_solve_graph(fmmlu_factor_h f, int32_t enable);

/* x = A_f^{-H} b (conjugate transpose of the factored inverse; same layout as fmmlu_solve). */
fmmlu_status fmmlu_solve_adjoint(fmmlu_factor_h f, const void* b, void* x, int64_t nrhs,
                                 void* hip_stream);

/*
 * Exact float64 product with the scaled system matrix, entries generated on the fly
 * (Section 3, eq. disc3): op 0: y = A~ x; 1: y = A~^H x; 2: y = (dA~/dk) x; 3: y = (dA~/deta) x.
 * x, y: device complex128 vectors of length n, original point order; must not alias.
 */
fmmlu_status fmmlu_matvec(fmmlu_factor_h f, int32_t op, const void* x, void* y, void* hip_stream);

/*
 * Allocation-free variant of fmmlu_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operation, arguments and kernels as fmmlu_matvec, but its scratch (the permuted
 * input, the tree-order result and the source-slice partial sums: (2 + s) * n complex128
 * entries, 1 <= s <= 16 slices) lives in a static device array of 64 MiB (4,194,304
 * entries) that the library holds on each GPU it runs on until the process ends; nothing
 * is allocated or freed. The slice count is limited so that the scratch fits, which it does
 * for n up to 1,398,101 (one slice); a larger n returns FMMLU_EINVAL. The current device must be the factor's device (EINVAL
 * otherwise). Asynchronous on hip_stream (no synchronisation). Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (different streams or
 * host threads) race and must be serialised by the caller.
 */
fmmlu_status fmmlu_matvec_noalloc(fmmlu_factor_h f, int32_t op, const void* x, void* y, void* hip_stream);

/*
 * Far-field pattern operator (Section 6.3's far-field pattern F[u], defined by
 * u(x) = e^{ikr}/r F(x^) + O(1/r^2), of the potential u = sum_j K(x, x_j) sqrt(w_j) sigma~_j;
 * the form below follows from the large-|x| limit of K):
 *     C[m, j] = (-i / 4 pi) sqrt(w_j) (k d_m.n_j + eta) e^{-ik d_m.x_j}.
 * dirs: DEVICE float64 SoA 3*ndir unit directions d_m (d_x[0..ndir), d_y, d_z).
 * op 0: out (ndir) = C in (n);  1: out (n) = C^H in (ndir);
 * op 2: out (ndir) = (dC/dk) in (n);  3: out (ndir) = (dC/deta) in (n).
 * in, out: device complex128, vectors of length n in the original point order; must not
 * alias. Sums are taken in a fixed order (deterministic). Synchronises the stream.
 */
fmmlu_status fmmlu_farfield(fmmlu_factor_h f, const double* dirs, int64_t ndir, int32_t op,
                            const void* in, void* out, void* hip_stream);

/*
 * Iterative refinement (Section 7's use of a low-precision direct solver as a
 * preconditioner): right-preconditioned restarted GMRES in float64 on A~ (adjoint != 0:
 * on A~^H) with the exact matvec above, preconditioned by fmmlu_solve (fmmlu_solve_adjoint).
 * b, x: device complex128 vectors of length n. x is overwritten. Starts from x0 = 0 (the
 * first step applies the factored inverse to b); each iteration is one factored-inverse
 * application and one exact product. Stops when the true residual, recomputed with the
 * exact product after each restart cycle or reached tolerance, satisfies
 * ||b - A~ x|| <= tol ||b||, or after maxit iterations (FMMLU_ENOCONV; *relres and *iters
 * still reported). Synchronises the stream.
 */
fmmlu_status fmmlu_solve_refined(fmmlu_factor_h f, const void* b, void* x, int32_t adjoint,
                                 double tol, int32_t maxit, int32_t* iters, double* relres,
                                 void* hip_stream);

/*
 * Batch of independent problems (many scatterers, each its own system A~_i of Section 3):
 * problem i has tree trees[i], host geometry xyz[i], normals[i], weights[i] (layouts as in
 * fmmlu_factor) and wavenumber k[i], coupling eta[i]; every problem uses *opts. The problems
 * are factored concurrently by nthreads host threads (0: min(count, 8)), each driving its own
 * HIP stream on the calling thread's current device, so that one problem's latency-bound
 * phases overlap another's. Errors name the failing problem. The batch owns its factors.
 */
fmmlu_status fmmlu_factor_batch(int32_t count, const fmmlu_tree_h* trees, const double* const* xyz,
                                const double* const* normals, const double* const* weights,
                                const double* k, const double* eta, const fmmlu_opts* opts,
                                int32_t nthreads, fmmlu_batch_h* out);

/* Problem count and offsets[0..count] of each problem's unknowns in the concatenated vectors
 * of fmmlu_batch_solve (offsets[count] = total). Either pointer may be NULL. */
fmmlu_status fmmlu_batch_info(fmmlu_batch_h b, int32_t* count, int64_t* offsets);

/* Borrowed handle of problem i's factorization (for matvec, info, single solves); it stays
 * owned by the batch: do not pass it to fmmlu_factor_destroy. */
fmmlu_status fmmlu_batch_factor(fmmlu_batch_h b, int32_t i, fmmlu_factor_h* out);

/*
 * x_i = A_i^{-1} b_i (adjoint != 0: A_i^{-H} b_i) for every problem, on concatenated device
 * complex128 vectors of the batch's total length (problem i at offsets[i], original point
 * order). The sweeps of all problems replay from one captured HIP graph with a branch per
 * problem (captured on first use per direction). b and x may alias. Asynchronous on hip_stream.
 */
fmmlu_status fmmlu_batch_solve(fmmlu_batch_h b, const void* rhs, void* x, int32_t adjoint,
                               void* hip_stream);

void fmmlu_batch_destroy(fmmlu_batch_h b);

/* Statistics of a finished factorization. */
fmmlu_status fmmlu_factor_info(fmmlu_factor_h f, fmmlu_info* out);

/*
 * Per-box record of the factorization for inspection, in elimination order.
 * fmmlu_factor_boxes(f, &count, NULL, ...) returns the count in *count. Otherwise, for record r:
 * level[r], coord[3r..3r+2], m[r] (active DOFs), s[r] (skeleton size). skel, when not
 * NULL, receives for all records the skeleton DOFs as original point indices, sorted,
 * concatenated in record order (sum of s entries).
 */
fmmlu_status fmmlu_factor_boxes(fmmlu_factor_h f, int64_t* count, int32_t* level, int32_t* coord,
                                int32_t* m, int32_t* s, int64_t* skel);

/*
 * Factors of record rec (0 <= rec < count of fmmlu_factor_boxes, elimination order), copied
 * to host memory for inspection and testing (synchronises the device). sizes[0..2] receive
 * r = |R|, s = |S| and s + n_N. DOF lists as original point indices: R (r entries) and S (s)
 * in the order of the box's ID pivots, SN (s + n_N) = S followed by the near DOFs. Matrices,
 * complex128 column-major (widened when the factorization stores complex float32):
 *   T  (s x r)        interpolation matrix of the ID, A_{.R} ~ A_{.S} T (Section 4.1);
 *   Xi (r x r)        X_RR^{-1}, the inverse pivot block;
 *   L  ((s+n_N) x r)  X_{(S u N) R} X_RR^{-1};
 *   UT ((s+n_N) x r)  U^T with U = X_RR^{-1} X_{R (S u N)}.
 * Any output pointer may be NULL (call with only sizes first to size the buffers).
 * Errors: ESTATE (NULL factor), EINVAL (rec out of range), EHIP.
 */
fmmlu_status fmmlu_factor_box_data(fmmlu_factor_h f, int64_t rec, int32_t* sizes, int64_t* R, int64_t* S,
                                   int64_t* SN, void* T, void* Xi, void* L, void* UT);

/*
 * Kernel-class profile of the factorization (only when opts.profile was set): for each of
 * the FMMLU_NKCLASS classes (0 tile assembly, 1 ID-matrix generation, 2 Householder QR,
 * 3 pivoted QR, 4 elimination GEMMs and gathers, 5 pivot-block inversion, 6 Schur update,
 * 7 top block), ms[c] is the GPU time summed over HIP-event-bracketed launches on the
 * factorization stream, launches[c] the number of brackets, flops[c] and bytes[c] the
 * algorithmic work (complex multiply-add = 8 flops). Host arrays of FMMLU_NKCLASS entries;
 * any may be NULL.
 */
#define FMMLU_NKCLASS 8
fmmlu_status fmmlu_factor_profile(fmmlu_factor_h f, double* ms, int64_t* launches, double* flops,
                                  double* bytes);

void fmmlu_factor_destroy(fmmlu_factor_h f);

/*
 * Kernel-block generation on the device (the entry generator the factorization uses):
 * out[i + j*nr] = A~[rows[i], cols[j]] for i < nr, j < nc, complex128, with the diagonal
 * value 1/2 where rows[i] == cols[j]. xyz, nrm: device SoA 3*n doubles; w: device n
 * doubles; rows, cols, out: device. For testing and for callers that assemble blocks.
 */
fmmlu_status fmmlu_kernel_block(const double* xyz, const double* nrm, const double* w, int64_t n,
                                double k, double eta, const int64_t* rows, int64_t nr,
                                const int64_t* cols, int64_t nc, void* out, void* hip_stream);

/*
 * Proxy rows on the device (the generator the factorization uses for the ID matrix, Sections
 * 5.1.1-5.1.3): with y_l = centre + radius u_l (l < ngamma), u_l the Fibonacci lattice of the
 * unit sphere (z_l = 1 - (2l+1)/ngamma, phi_l = l pi (3 - sqrt 5)) and s = sqrt(4 pi radius^2 /
 * ngamma), out (2 ngamma x m, complex128 column-major) holds
 *   rows l < ngamma:        s K(y_l, x_j) sqrt(w_j)   (outgoing, source normal n_j),
 *   rows ngamma + l:        s G(x_j, y_l) sqrt(w_j)   (incoming, single layer),
 * for columns j = dofs[0..m) (device int64, original point indices). xyz, nrm: device SoA
 * 3*n doubles; w: device n doubles; centre: host 3 doubles. For testing and for callers that
 * build ID matrices. Errors: EINVAL (NULL pointers, sizes, index out of range), ENOMEM, EHIP.
 * Synchronises the stream.
 */
fmmlu_status fmmlu_proxy_block(const double* xyz, const double* nrm, const double* w, int64_t n, double k,
                               double eta, const int64_t* dofs, int64_t m, const double* centre, double radius,
                               int32_t ngamma, void* out, void* hip_stream);

/*
 * Batched dense inverse with partial pivoting (blocked Gauss-Jordan), the routine that
 * inverts the pivot blocks X_RR (Section 4.1) and the top block (Section 4.2). a: device,
 * count consecutive n x n complex128 column-major matrices (not modified); out: device,
 * their inverses in the same layout. For testing and for callers that need dense inverses.
 * Errors: EINVAL, ESINGULAR (an exactly zero pivot), ENOMEM, EHIP. Synchronises the stream.
 */
fmmlu_status fmmlu_dense_inverse(const void* a, int64_t n, int64_t count, void* out, void* hip_stream);

/*
 * Frees the memory that released factorizations leave for reuse by later ones in the same
 * process: device blocks (factor storage, planning scratch, tile pools; at most 8 GiB) and
 * pinned host staging buffers (at most 512 MiB each for two pools). Call it between
 * factorizations, not while one is running on another thread. Errors: EHIP.
 */
fmmlu_status fmmlu_trim_caches(void);

/*
 * The GEMM autotuner's table for the current device (opts.gemm_autotune): for every use of the
 * batched GEMM (precision, mapped output, op(A)) and K bucket, the kernel chosen and the
 * measured milliseconds of each candidate on the synthetic batch, as a NUL-terminated JSON
 * object. buf: host, len bytes (may be NULL with len 0); *needed (may be NULL) receives the
 * bytes required including the NUL. ESTATE if no factorization has tuned the device yet;
 * EINVAL if len is too small (nothing written).
 */
fmmlu_status fmmlu_gemm_tuning(char* buf, int64_t len, int64_t* needed);

/* Message for the last non-OK status on this thread ("" if none). */
const char* fmmlu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMMLU_H */
