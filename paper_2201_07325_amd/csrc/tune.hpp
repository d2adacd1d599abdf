// GEMM autotuning (see tune.cpp): kernel choice per use and K bucket, measured once per device.
#pragma once

#include <string>

#include "common.hpp"
#include "kernels.hpp"

namespace fmmlu {

// K bucket of a batch whose longest product has inner dimension k
int gemm_bucket(int64_t k);
// the measured choice for this use and bucket on the current device (GK_AUTO before tuning),
// or the kernel forced on this thread (where it implements the use)
int gemm_tuned_kernel(bool c32, bool mapped, int opA, int64_t kmax);
// testing: every GEMM launched from this thread uses `kernel` (GK_AUTO: the tuned choice)
void gemm_force_kernel(int kernel);
// times every candidate kernel of every use and bucket on the current device (once per
// process; later calls return at once); scratch from mem, work on st (synchronous)
void gemm_autotune(DeviceMemory& mem, hipStream_t st);
// the current device's table as JSON ("" before tuning)
std::string gemm_tune_report();

}  // namespace fmmlu
