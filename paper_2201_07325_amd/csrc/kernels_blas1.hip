// Vector kernels of the float64 refinement: partial inner products with a fixed partition
// (deterministic sums), axpy, scaled copy, difference.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fmmlu {

namespace {

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(256) dotc_partial_kernel(const zd* __restrict__ x, const zd* __restrict__ y,
                                                           int64_t n, zd* __restrict__ part) {
  __shared__ zd red[4];
  zd acc{0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    zfmac(acc, x[i], y[i]);
  acc.re = wave_sum(acc.re);
  acc.im = wave_sum(acc.im);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = zadd(zadd(red[0], red[1]), zadd(red[2], red[3]));
}

__global__ void __launch_bounds__(256) axpy_kernel(zd a, const zd* __restrict__ x, zd* __restrict__ y,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) zfma(y[i], a, x[i]);
}

__global__ void __launch_bounds__(256) scal_copy_kernel(zd a, const zd* __restrict__ x, zd* __restrict__ y,
                                                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = zmul(a, x[i]);
}

__global__ void __launch_bounds__(256) sub_kernel(const zd* __restrict__ a, const zd* __restrict__ b,
                                                  zd* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = zsub(a[i], b[i]);
}

}  // namespace

void launch_dotc_partial(const zd* x, const zd* y, int64_t n, zd* part, hipStream_t st) {
  hipLaunchKernelGGL(dotc_partial_kernel, dim3(kDotBlocks), dim3(256), 0, st, x, y, n, part);
  FMMLU_HIP(hipGetLastError());
}

void launch_axpy(zd a, const zd* x, zd* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, x, y, n);
  FMMLU_HIP(hipGetLastError());
}

void launch_scal_copy(zd a, const zd* x, zd* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scal_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, x, y, n);
  FMMLU_HIP(hipGetLastError());
}

void launch_sub(const zd* a, const zd* b, zd* out, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(sub_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, out, n);
  FMMLU_HIP(hipGetLastError());
}

}  // namespace fmmlu
