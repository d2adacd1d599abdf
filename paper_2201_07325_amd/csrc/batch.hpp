// Solves of a batch of independent factorizations: one HIP graph per direction with a
// branch per problem (the problems' sweeps run concurrently), on concatenated vectors.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "factor.hpp"

namespace fmmlu {

class BatchSolver {
 public:
  void init(const std::vector<FactorImpl*>& fs, const std::vector<int64_t>& offsets);
  // x = A_i^{-1} b (or A_i^{-H} b) for every problem i, on the concatenated vectors
  void solve(const zd* b, zd* x, bool adjoint, hipStream_t st);
  ~BatchSolver();

 private:
  bool capture(int adj);
  std::vector<FactorImpl*> fs_;
  std::vector<int64_t> off_;
  DeviceArena arena_{size_t(1) << 20};
  zd* gin_ = nullptr;
  zd* gout_ = nullptr;
  hipStream_t cap_ = nullptr;
  std::vector<hipStream_t> branch_;
  std::vector<hipEvent_t> ev_;
  hipGraph_t graph_[2] = {nullptr, nullptr};
  hipGraphExec_t exec_[2] = {nullptr, nullptr};
  bool use_graph_ = true;
};

}  // namespace fmmlu
