// Factorization object: recursive strong skeletonization driven level by level from the
// host, every arithmetic step in device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "tree.hpp"

namespace fmmlu {

// Pinned host staging memory for task descriptors; bump allocation, reset after a sync.
// frees the device and pinned host memory that finished factorizations left for reuse
void trim_reuse_caches();

class HostStage {
 public:
  ~HostStage();
  void* alloc(size_t bytes);
  void reset() {
    cur_ = 0;
    used_ = 0;
  }

 private:
  std::vector<void*> chunks_;
  std::vector<size_t> sizes_;
  size_t cur_ = 0, used_ = 0;
};

// Opt-in timing of kernel classes with HIP events on the launch stream. Algorithmic work
// (flops or bytes, per class) is accumulated by the caller alongside.
enum KClass { KC_ASSEMBLE = 0, KC_IDMAT, KC_QR, KC_CPQR, KC_ELIM, KC_INV, KC_SCHUR, KC_TOP, KC_COUNT };
struct Profiler {
  bool on = false;
  unsigned mask = ~0u;  // classes bracketed while on
  hipStream_t st = nullptr;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> open;
  std::vector<hipEvent_t> free_ev;
  double ms[KC_COUNT] = {0};
  int64_t launches[KC_COUNT] = {0};
  double flops[KC_COUNT] = {0};
  double bytes[KC_COUNT] = {0};
  int cur = -1;
  hipEvent_t cur_a = nullptr;
  hipEvent_t get();
  void begin(int cls);
  void end();
  void harvest();  // after a stream synchronisation
  ~Profiler();
};
struct ProfScope {
  Profiler& p;
  ProfScope(Profiler& pr, int cls) : p(pr) { p.begin(cls); }
  ~ProfScope() { p.end(); }
};

struct FactorBox {
  int level, box;
  int coord[3];
  int m, s, r, nsn;
  int64_t y_off;
  std::vector<int64_t> skel_orig;  // skeleton DOFs as original indices (sorted)
  SolveBox dev;                    // device pointers and sizes
};

struct SolvePhase {
  int box_begin = 0, box_end = 0;  // range in boxes
  SolveBox* dboxes = nullptr;      // device array
  int32_t* sc_dst = nullptr;       // scatter CSR: destination tree positions
  int64_t* sc_ptr = nullptr;
  int64_t* sc_src = nullptr;
  int64_t nd = 0;
  int direct = 0;  // every scatter destination has one contribution: y goes straight into x
  int64_t ylen = 0, plen = 0, xrplen = 0;
  // counts of the work items of 64 (forward x_R partials, rows of y; backward x_R partials,
  // rows of x_S), from which each sweep picks its granularity
  int nxr = 0, ny = 0, nbp = 0, nbt = 0;
  SweepTask* dbt16 = nullptr;  // blocked sweeps: rows of x_S in items of 16
  int nbt16 = 0;
  // the same steps, each in items of 64 or of 16 outputs / rows (g1*), for the single-vector
  // sweeps and (all but the rows of x_S) the blocked ones
  SweepTask *s1xr = nullptr, *s1y = nullptr, *s1bp = nullptr, *s1bt = nullptr;
  int n1xr = 0, n1y = 0, n1bp = 0, n1bt = 0;
  int g1xr = kSolveOut, g1y = kSolveRows, g1bp = kSolveOut, g1bt = kSolveRows;
  // blocked sweeps: backward x_R summed once per phase (items of 64 entries of R) where the
  // 16-row items would each re-read many partials
  SweepTask* dxs = nullptr;
  int nxs = 0, blk_presum = 0;
  int rmax = 0, smax = 0;
};

// Workspace of the sweeps for blocks of nr right-hand sides (interleaved vectors)
struct SolveWs {
  zd *x = nullptr, *y = nullptr, *top = nullptr, *p = nullptr, *xrp = nullptr;
  zd* xrg = nullptr;  // x_R of every box (offset dx_off) after the forward sweep
  zd* xrd = nullptr;  // the same with D^{-1} applied
};

struct FactorImpl {
  int64_t n = 0;
  double k = 0, eta = 0;
  bool f32 = false;  // tiles and stored factors in complex float32
  fmmlu_opts opts{};
  int device = 0;
  // every device block of the factorization (declared before the arenas that return to it)
  DeviceMemory mem;
  DeviceArena arena;  // persistent: geometry, factors, top
  double* geom = nullptr;
  int64_t* order_dev = nullptr;  // tree position -> original index
  DevGeom g{};
  std::vector<int64_t> order;  // host copy
  std::vector<FactorBox> boxes;
  std::vector<SolvePhase> phases;
  int64_t ymax = 0, pmax = 0, xrpmax = 0;
  SolveBox* all_boxes = nullptr;  // every factored box, for the diagonal step
  int nall = 0, rmax_all = 0;
  SweepTask* dg_tasks = nullptr;  // diagonal step: (box of all_boxes, 64 outputs)
  int ndg = 0;
  int64_t dxlen = 0;  // x_R of every box in one buffer (sum of r)
  int n0 = 0;
  int32_t* top_dev = nullptr;
  zd* Ainv = nullptr;
  fmmlu_info info{};
  Profiler prof;
  // solve workspace (allocated lazily)
  SolveWs ws1{};        // single right-hand sides
  zd* wmv = nullptr;
  zd* wpart = nullptr;  // matvec slice partials
  int64_t wpart_entries = 0;
  // refinement workspace (allocated on the first refined solve)
  DeviceArena rarena{size_t(1) << 20};
  zd* rbuf = nullptr;
  // far-field partial sums (grown on demand)
  DeviceArena farena{size_t(1) << 20};
  zd* fpart = nullptr;
  int64_t fpart_cap = 0;

  void factor(const Octree& tree, const double* xyz, const double* nrm, const double* w,
              hipStream_t st);
  void solve(const zd* b, zd* x, int64_t nrhs, bool adjoint, hipStream_t st);
  // one right-hand side, every kernel of the sweeps (no copies, no allocation)
  void solve_core(const zd* b, zd* x, bool adjoint, hipStream_t st);
  // the sweeps for m <= nr right-hand sides (columns of b and x at strides ldb, ldx)
  void sweep(const SolveWs& w, int nr, const zd* b, int64_t ldb, zd* x, int64_t ldx, int m, bool adjoint,
             hipStream_t st);
  void ensure_workspace();
  void alloc_ws(SolveWs& w, int nr);
  // blocks of kSolveBlock right-hand sides (allocated on the first multi-column solve)
  SolveWs wsb{};
  zd* ginb = nullptr;
  zd* goutb = nullptr;
  hipGraph_t graphb[2] = {nullptr, nullptr};
  hipGraphExec_t gexecb[2] = {nullptr, nullptr};
  bool blocked_ok() const;
  void ensure_block_workspace();
  bool capture_block(int adj);
  // solves replay a captured HIP graph per direction (input/output through gin/gout)
  bool use_graph = true;
  bool precapture = true;  // capture the solve graphs while the top block runs (single factorizations)
  hipStream_t gstream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  zd* gin = nullptr;
  zd* gout = nullptr;
  bool capture(int adj);
  ~FactorImpl();
  // exact float64 product in the original point order (op as fmmlu_matvec)
  void matvec(int op, const zd* x, zd* y, hipStream_t st);
  // restarted right-preconditioned FGMRES; returns true when relres <= tol
  bool refine(const zd* b, zd* x, bool adjoint, double tol, int maxit, int* iters, double* relres,
              hipStream_t st);
};

// inverses of count consecutive n x n column-major matrices (device memory, A preserved)
void dense_inverse_batch(const zd* A, int64_t n, int64_t count, zd* out, hipStream_t st);

}  // namespace fmmlu
