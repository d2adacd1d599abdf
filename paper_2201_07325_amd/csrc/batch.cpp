// Batched solves over independent factorizations (see batch.hpp).
#include "batch.hpp"

namespace fmmlu {

void BatchSolver::init(const std::vector<FactorImpl*>& fs, const std::vector<int64_t>& offsets) {
  fs_ = fs;
  off_ = offsets;
  for (auto* f : fs_) f->ensure_workspace();
  const int64_t total = off_.back();
  gin_ = arena_.alloc_n<zd>((size_t)total);
  gout_ = arena_.alloc_n<zd>((size_t)total);
}

// The capture stream forks one branch per problem (event wait), each branch replays that
// problem's sweeps on its own workspace, and the branches join back before the end.
bool BatchSolver::capture(int adj) {
  if (exec_[adj]) return true;
  const size_t nb = fs_.size();
  if (!cap_) {
    FMMLU_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
    branch_.resize(nb, nullptr);
    for (auto& s : branch_) FMMLU_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ev_.resize(nb + 1, nullptr);
    for (auto& e : ev_) FMMLU_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = hipEventRecord(ev_[nb], cap_) == hipSuccess;
  try {
    for (size_t i = 0; ok && i < nb; ++i) {
      ok = hipStreamWaitEvent(branch_[i], ev_[nb], 0) == hipSuccess;
      if (!ok) break;
      fs_[i]->solve_core(gin_ + off_[i], gout_ + off_[i], adj != 0, branch_[i]);
      ok = hipEventRecord(ev_[i], branch_[i]) == hipSuccess && hipStreamWaitEvent(cap_, ev_[i], 0) == hipSuccess;
    }
  } catch (const Error&) {
    ok = false;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cap_, &g);
  if (e != hipSuccess || !ok || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return false;
  }
  graph_[adj] = g;
  exec_[adj] = x;
  return true;
}

void BatchSolver::solve(const zd* b, zd* x, bool adjoint, hipStream_t st) {
  const int adj = adjoint ? 1 : 0;
  const size_t bytes = sizeof(zd) * (size_t)off_.back();
  if (use_graph_ && !capture(adj)) use_graph_ = false;
  FMMLU_HIP(hipMemcpyAsync(gin_, b, bytes, hipMemcpyDeviceToDevice, st));
  if (use_graph_) {
    FMMLU_HIP(hipGraphLaunch(exec_[adj], st));
  } else {
    for (size_t i = 0; i < fs_.size(); ++i) fs_[i]->solve_core(gin_ + off_[i], gout_ + off_[i], adjoint, st);
  }
  FMMLU_HIP(hipMemcpyAsync(x, gout_, bytes, hipMemcpyDeviceToDevice, st));
}

BatchSolver::~BatchSolver() {
  for (int a = 0; a < 2; ++a) {
    if (exec_[a]) (void)hipGraphExecDestroy(exec_[a]);
    if (graph_[a]) (void)hipGraphDestroy(graph_[a]);
  }
  for (auto e : ev_)
    if (e) (void)hipEventDestroy(e);
  for (auto s : branch_)
    if (s) (void)hipStreamDestroy(s);
  if (cap_) (void)hipStreamDestroy(cap_);
}

}  // namespace fmmlu
