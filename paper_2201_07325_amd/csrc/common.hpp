// Shared host/device definitions of the FMM-LU library: complex arithmetic, error
// handling, and a bump-pointer device arena.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/fmmlu.h"

namespace fmmlu {

// ---------------------------------------------------------------------------------
// complex float64 (interleaved, 16-byte aligned; same layout as std::complex<double>)
struct alignas(16) zd {
  double re, im;
};
struct alignas(8) zf {
  float re, im;
};

__host__ __device__ inline zd zmake(double r, double i) { return zd{r, i}; }
// storage conversions between complex float64 and float32
__host__ __device__ inline zd widen(zd v) { return v; }
__host__ __device__ inline zd widen(zf v) { return zd{(double)v.re, (double)v.im}; }
template <class T>
__host__ __device__ inline T narrow(zd v);
template <>
__host__ __device__ inline zd narrow<zd>(zd v) {
  return v;
}
template <>
__host__ __device__ inline zf narrow<zf>(zd v) {
  return zf{(float)v.re, (float)v.im};
}
__host__ __device__ inline zd zadd(zd a, zd b) { return zd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline zd zsub(zd a, zd b) { return zd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline zd zmul(zd a, zd b) {
  return zd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline zd zconj(zd a) { return zd{a.re, -a.im}; }
__host__ __device__ inline zd zscale(zd a, double s) { return zd{a.re * s, a.im * s}; }
__host__ __device__ inline double zabs2(zd a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
__host__ __device__ inline void zfma(zd& acc, zd a, zd b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += conj(a) * b
__host__ __device__ inline void zfmac(zd& acc, zd a, zd b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}
__host__ __device__ inline zd zdiv(zd a, zd b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return zd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    double r = b.re / b.im, d = b.im + b.re * r;
    return zd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}

// ---------------------------------------------------------------------------------
// errors: thrown inside the library, converted to fmmlu_status at the C boundary
struct Error : std::runtime_error {
  fmmlu_status status;
  Error(fmmlu_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define FMMLU_HIP(call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::fmmlu::Error(FMMLU_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define FMMLU_REQUIRE(cond, status, msg)                        \
  do {                                                          \
    if (!(cond)) throw ::fmmlu::Error(status, std::string(msg)); \
  } while (0)

// ---------------------------------------------------------------------------------
// Device memory blocks given back by one factorization and taken by the next (hipMalloc and
// hipFree of large blocks cost a fraction of a millisecond each, and hipFree waits for the
// device). A block is given back with an event recorded on the stream that last used it, and
// take() waits for that event before handing the block out, so a block is never reused while
// queued work may still read or write it. At most kMax bytes are kept; the cache is never torn
// down (the process exit reclaims the memory; fmmlu_trim_caches frees it earlier).
class DeviceChunkCache {
 public:
  static constexpr size_t kMax = size_t(8) << 30;
  static DeviceChunkCache& get() {
    static DeviceChunkCache* c = new DeviceChunkCache;
    return *c;
  }
  // smallest cached block of the current device holding at least b bytes (its size in cap)
  void* take(size_t b, size_t& cap) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    Block blk{};
    {
      std::lock_guard<std::mutex> l(m_);
      int best = -1;
      for (int i = 0; i < (int)free_.size(); ++i)
        if (free_[i].dev == dev && free_[i].cap >= b && (best < 0 || free_[i].cap < free_[best].cap)) best = i;
      if (best < 0) return nullptr;
      blk = free_[best];
      held_ -= blk.cap;
      free_.erase(free_.begin() + best);
    }
    if (blk.ev) {
      const hipError_t e = hipEventSynchronize(blk.ev);
      (void)hipEventDestroy(blk.ev);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(blk.p);
        return nullptr;
      }
    }
    cap = blk.cap;
    return blk.p;
  }
  // free every cached block (of every device)
  void trim() {
    std::vector<Block> all;
    {
      std::lock_guard<std::mutex> l(m_);
      all.swap(free_);
      held_ = 0;
    }
    for (auto& b : all) {
      if (b.ev) {
        (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
      }
      (void)hipFree(b.p);
    }
  }
  // give a block back; st is the stream whose queued work may still use it
  void give(void* p, size_t cap, hipStream_t st) {
    int dev = 0;
    hipEvent_t ev = nullptr;
    if (hipGetDevice(&dev) == hipSuccess && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
      if (hipEventRecord(ev, st) == hipSuccess) {
        std::lock_guard<std::mutex> l(m_);
        if (held_ + cap <= kMax) {
          free_.push_back(Block{p, cap, dev, ev});
          held_ += cap;
          return;
        }
      }
      (void)hipEventDestroy(ev);
    }
    (void)hipGetLastError();
    (void)hipFree(p);  // hipFree waits for the device
  }

 private:
  struct Block {
    void* p;
    size_t cap;
    int dev;
    hipEvent_t ev;
  };
  std::mutex m_;
  std::vector<Block> free_;
  size_t held_ = 0;
};

// Every device block one factorization holds comes from, and goes back to, its DeviceMemory:
// the caller's allocator when one is given (fmmlu_opts.alloc / free / alloc_ctx), else
// hipMalloc with the process-wide DeviceChunkCache. It counts the bytes held (peak_bytes)
// and enforces the device memory cap on that count. Blocks go back only once the work that
// used them is finished or ordered before later work on the release stream.
class DeviceMemory {
 public:
  void configure(const fmmlu_opts& o, hipStream_t st) {
    ualloc_ = o.alloc;
    ufree_ = o.free;
    uctx_ = o.alloc_ctx;
    cap_ = o.device_mem_cap > 0 ? (size_t)o.device_mem_cap : 0;
    st_ = st;
  }
  // stream on which later releases are ordered (the null stream once the factorization's own
  // stream may be gone)
  void set_stream(hipStream_t st) { st_ = st; }
  hipStream_t stream() const { return st_; }
  // at least `bytes` bytes; the block's size in `got`. Throws ENOMEM.
  void* get(size_t bytes, size_t& got) {
    if (bytes == 0) bytes = 256;
    {
      std::lock_guard<std::mutex> l(m_);
      if (cap_ && held_ + bytes > cap_)
        throw Error(FMMLU_ENOMEM, "device memory cap exceeded (" + std::to_string(held_ + bytes) + " > " +
                                      std::to_string(cap_) + " bytes)");
    }
    void* p = nullptr;
    got = bytes;
    if (ualloc_) {
      p = ualloc_(bytes, st_, uctx_);
      if (!p) throw Error(FMMLU_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
      if (!cap_) p = DeviceChunkCache::get().take(bytes, got);  // a cap counts exact sizes
      if (!p) {
        got = bytes;
        const hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          throw Error(FMMLU_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
      }
    }
    std::lock_guard<std::mutex> l(m_);
    held_ += got;
    peak_ = held_ > peak_ ? held_ : peak_;
    return p;
  }
  void put(void* p, size_t got) {
    if (!p) return;
    {
      std::lock_guard<std::mutex> l(m_);
      held_ -= got;
    }
    if (ufree_)
      ufree_(p, st_, uctx_);
    else
      DeviceChunkCache::get().give(p, got, st_);
  }
  // blocks allocated elsewhere but held for this factorization (counted and capped only)
  void account(size_t bytes) {
    std::lock_guard<std::mutex> l(m_);
    if (cap_ && held_ + bytes > cap_)
      throw Error(FMMLU_ENOMEM, "device memory cap exceeded (" + std::to_string(held_ + bytes) + " > " +
                                    std::to_string(cap_) + " bytes)");
    held_ += bytes;
    peak_ = held_ > peak_ ? held_ : peak_;
  }
  void unaccount(size_t bytes) {
    std::lock_guard<std::mutex> l(m_);
    held_ -= bytes;
  }
  size_t held() const { return held_; }
  size_t peak() const { return peak_; }
  bool caller_allocator() const { return ualloc_ != nullptr; }

 private:
  void* (*ualloc_)(size_t, void*, void*) = nullptr;
  void (*ufree_)(void*, void*, void*) = nullptr;
  void* uctx_ = nullptr;
  size_t cap_ = 0;
  hipStream_t st_ = nullptr;
  std::mutex m_;
  size_t held_ = 0, peak_ = 0;
};

// Device arena: large chunks, bump allocation, 256-byte alignment, freed together. Chunks come
// from a DeviceMemory when one is attached (counted, capped, recycled), else straight from
// hipMalloc (stand-alone utilities).
class DeviceArena {
 public:
  explicit DeviceArena(size_t chunk = size_t(256) << 20, DeviceMemory* mem = nullptr) : chunk_(chunk), mem_(mem) {}
  ~DeviceArena() { release(); }
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;

  void* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (cur_ < chunks_.size() && used_ + bytes <= sizes_[cur_]) {
      void* p = static_cast<char*>(chunks_[cur_]) + used_;
      used_ += bytes;
      total_ += bytes;
      return p;
    }
    // advance to the next existing chunk that fits, else allocate a new one
    while (cur_ + 1 < chunks_.size()) {
      ++cur_;
      used_ = 0;
      if (bytes <= sizes_[cur_]) return alloc(bytes);
    }
    size_t sz = bytes > chunk_ ? bytes : chunk_;
    void* p = nullptr;
    if (mem_) {
      p = mem_->get(sz, sz);
    } else {
      const hipError_t e = hipMalloc(&p, sz);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(FMMLU_ENOMEM, "hipMalloc of " + std::to_string(sz) + " bytes failed");
      }
    }
    chunks_.push_back(p);
    sizes_.push_back(sz);
    held_ += sz;
    cur_ = chunks_.size() - 1;
    used_ = 0;
    return alloc(bytes);
  }
  template <class T>
  T* alloc_n(size_t n) {
    return static_cast<T*>(alloc(n * sizeof(T)));
  }
  // forget all allocations but keep the chunks for reuse
  void reset() {
    cur_ = 0;
    used_ = 0;
    total_ = 0;
  }
  void release() {
    for (size_t i = 0; i < chunks_.size(); ++i) {
      if (mem_)
        mem_->put(chunks_[i], sizes_[i]);
      else
        (void)hipFree(chunks_[i]);
    }
    chunks_.clear();
    sizes_.clear();
    cur_ = 0;
    used_ = 0;
    held_ = 0;
    total_ = 0;
  }
  size_t held() const { return held_; }
  void set_chunk(size_t c) { chunk_ = c; }
  void set_memory(DeviceMemory* m) { mem_ = m; }

 private:
  size_t chunk_;
  DeviceMemory* mem_ = nullptr;
  std::vector<void*> chunks_;
  std::vector<size_t> sizes_;
  size_t cur_ = 0, used_ = 0, held_ = 0, total_ = 0;
};

}  // namespace fmmlu
