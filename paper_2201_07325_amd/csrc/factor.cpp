// Recursive strong skeletonization (Sections 4.1-4.4, 5.1-5.2), driven level by level.
//
// Storage ("pair tiles"). At level l every active DOF is owned by its level-l box or, when
// its leaf is coarser, by that leaf. For every ordered pair of owners whose L-infinity gap
// is at most one side of the finer of the two, the block A[act(o1), act(o2)] is kept as a
// dense column-major tile. Schur-complement updates only ever touch such pairs (two boxes
// that both touch the box being eliminated are at most one box apart), and every other
// entry is still a pure kernel value (Section 4.4's invariant), so it is regenerated on
// demand instead of stored.
//
// Per level: tiles are assembled (copied from the previous level's tiles restricted to the
// surviving skeletons, or generated), then the level's boxes are processed in eight colour
// phases (parity of the integer box coordinates), each phase as one concurrent step: every
// box classifies the DOFs that are live when the phase begins. Same-colour boxes never touch,
// so no box's elimination reads a block another box of its phase writes, and their Schur
// updates to shared near-near tiles are summed by one output-stationary GEMM task per
// destination tile. Two same-colour boxes can lie in each other's Q region, though: the Q
// rows of one then still hold the other's redundant DOFs, rows that its own ID has shown to
// be combinations of its skeleton rows to the tolerance, so both IDs stay valid.
// Within a phase:
//   1. ID matrix M = [A_QB ; A_BQ^T ; proxy outgoing ; proxy incoming]  (Section 5.1.3)
//   2. greedy CPQR of M -> S, R, T (Section 4.1): pivoted Cholesky of the Gram matrix M^H M
//      (eps >= 1e-7), or blocked Householder QR of M then column pivoting on R
//   3. gathers and GEMMs for X_RR, X_{(S u N) R}, X_{R (S u N)}       (Section 4.1)
//   4. Gauss-Jordan inversion of X_RR, panels L = X_{.R} X_RR^{-1}, U = X_RR^{-1} X_{R.}
//   5. Schur update of the near-near tiles with X_{.R} U
// The host only plans (index lists, task descriptors) and reads back ranks and pivots.
#include "factor.hpp"
#include "tune.hpp"

#include <algorithm>
#include <atomic>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>

namespace fmmlu {

// ------------------------------------------------------------------------------------------
// Pinned host staging blocks outlive the factorization that allocated them: later ones take
// them back instead of pinning new memory. At most kMax bytes are kept; never torn down (no
// HIP calls at static teardown; the process exit reclaims the memory).
class PinnedCache {
 public:
  static constexpr size_t kMax = size_t(512) << 20;
  static PinnedCache& get() {
    static PinnedCache* c = new PinnedCache;
    return *c;
  }
  void* take(size_t b, size_t& cap) {
    std::lock_guard<std::mutex> l(m_);
    int best = -1;
    for (int i = 0; i < (int)free_.size(); ++i)
      if (free_[i].second >= b && (best < 0 || free_[i].second < free_[best].second)) best = i;
    if (best < 0) return nullptr;
    void* p = free_[best].first;
    cap = free_[best].second;
    held_ -= cap;
    free_.erase(free_.begin() + best);
    return p;
  }
  void trim() {
    std::vector<std::pair<void*, size_t>> all;
    {
      std::lock_guard<std::mutex> l(m_);
      all.swap(free_);
      held_ = 0;
    }
    for (auto& b : all) (void)hipHostFree(b.first);
  }
  void give(void* p, size_t cap) {
    {
      std::lock_guard<std::mutex> l(m_);
      if (held_ + cap <= kMax) {
        free_.emplace_back(p, cap);
        held_ += cap;
        return;
      }
    }
    (void)hipHostFree(p);
  }

 private:
  std::mutex m_;
  std::vector<std::pair<void*, size_t>> free_;
  size_t held_ = 0;
};

HostStage::~HostStage() {
  for (size_t i = 0; i < chunks_.size(); ++i) PinnedCache::get().give(chunks_[i], sizes_[i]);
}

void* HostStage::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (cur_ < chunks_.size()) {
    if (used_ + bytes <= sizes_[cur_]) {
      void* p = static_cast<char*>(chunks_[cur_]) + used_;
      used_ += bytes;
      return p;
    }
    ++cur_;
    used_ = 0;
  }
  size_t sz = std::max(bytes, size_t(64) << 20);
  void* p = PinnedCache::get().take(bytes, sz);
  if (!p) FMMLU_HIP(hipHostMalloc(&p, sz, hipHostMallocDefault));
  chunks_.push_back(p);
  sizes_.push_back(sz);
  cur_ = chunks_.size() - 1;
  used_ = bytes;
  return p;
}

hipEvent_t Profiler::get() {
  if (!free_ev.empty()) {
    hipEvent_t e = free_ev.back();
    free_ev.pop_back();
    return e;
  }
  hipEvent_t e;
  FMMLU_HIP(hipEventCreate(&e));
  return e;
}
void Profiler::begin(int cls) {
  if (!on || !((mask >> cls) & 1u)) return;
  cur = cls;
  cur_a = get();
  FMMLU_HIP(hipEventRecord(cur_a, st));
}
void Profiler::end() {
  if (!on || cur < 0) return;
  hipEvent_t b = get();
  FMMLU_HIP(hipEventRecord(b, st));
  open.push_back(Rec{cur, cur_a, b});
  launches[cur]++;
  cur = -1;
}
void Profiler::harvest() {
  if (!on) return;
  for (auto& r : open) {
    float t = 0.f;
    FMMLU_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    free_ev.push_back(r.a);
    free_ev.push_back(r.b);
  }
  open.clear();
}
Profiler::~Profiler() {
  for (auto& r : open) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : free_ev) (void)hipEventDestroy(e);
}

namespace {

using Clock = std::chrono::steady_clock;

// Tolerances at or above this use the Gram-matrix route to the greedy CPQR: pivoted
// Cholesky of M^H M has the same pivots and R as CPQR of M in exact arithmetic, and in
// float64 its error floor (~sqrt(u) relative to |M|) stays well below eps down to 1e-7.
constexpr double kGramEps = 1e-7;

struct Owner {
  int box = -1;
  int level = 0;
  int64_t c[3] = {0, 0, 0};
  int64_t first_pos = 0;        // first tree position of the box (ordering key)
  std::vector<int64_t> act;     // tree positions of the tile rows at this level
  std::vector<int32_t> live;    // positions in act still active (ascending)
  int32_t* live_dev = nullptr;  // device copy of live
  int32_t* perm_dev = nullptr;  // pivot order when processed at this level
  std::vector<int> sub;         // previous-level owners merged into this one
  std::vector<int64_t> sub_rowbase;
};

// gap between two owner boxes in units of the finer one's size (0: touching)
template <class O>
int64_t gap_units(const O& a, const O& b) {
  const int L = std::max(a.level, b.level);
  const int64_t sa = int64_t(1) << (L - a.level), sb = int64_t(1) << (L - b.level);
  int64_t g = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const int64_t alo = a.c[ax] * sa, ahi = (a.c[ax] + 1) * sa;
    const int64_t blo = b.c[ax] * sb, bhi = (b.c[ax] + 1) * sb;
    g = std::max(g, std::max(blo - ahi, alo - bhi));
  }
  return std::max<int64_t>(g, 0);
}

// Close owners of each owner (gap <= 1 box) in ascending order, with the offsets of their
// pair tiles in the level's tile pool.
struct PairIndex {
  std::vector<int64_t> beg{0};  // owner a's pairs: [beg[a], beg[a + 1])
  std::vector<int32_t> ids;
  std::vector<int64_t> off;
  int64_t pos(int a, int b) const {  // index of pair (a, b) in ids / off, or -1
    const auto first = ids.begin() + beg[a], last = ids.begin() + beg[a + 1];
    const auto it = std::lower_bound(first, last, b);
    return (it != last && *it == b) ? (int64_t)(it - ids.begin()) : -1;
  }
  int64_t find(int a, int b) const {  // offset of tile (a, b), or -1
    const int64_t k = pos(a, b);
    return k < 0 ? -1 : off[k];
  }
  int64_t at(int a, int b) const {
    const int64_t o = find(a, b);
    if (o < 0) throw Error(FMMLU_EINVAL, "internal: tile of a pair that is not close");
    return o;
  }
};

// Host worker threads kept for one factorization: ranges(n, grain, fn) runs fn(lo, hi) over
// contiguous ranges of [0, n) on the caller and the workers. fn must not throw.
class HostPool {
 public:
  explicit HostPool(int nworkers) : nw_(std::max(1, nworkers)) {
    for (int w = 1; w < nw_; ++w) th_.emplace_back([this, w] { loop(w); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> l(m_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  template <class F>
  void ranges(int n, int grain, F&& fn) {
    const int nt = std::max(1, std::min(nw_, n / std::max(grain, 1)));
    if (nt <= 1) {
      fn(0, n);
      return;
    }
    const int chunk = (n + nt - 1) / nt;
    std::function<void(int)> job = [&](int w) {
      const int lo = w * chunk, hi = std::min(n, lo + chunk);
      if (lo < hi) fn(lo, hi);
    };
    {
      std::lock_guard<std::mutex> l(m_);
      job_ = &job;
      nt_ = nt;
      left_ = nt - 1;
      ++gen_;
    }
    cv_.notify_all();
    job(0);
    std::unique_lock<std::mutex> l(m_);
    done_.wait(l, [&] { return left_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop(int w) {
    int64_t seen = 0;
    for (;;) {
      std::function<void(int)>* job = nullptr;
      {
        std::unique_lock<std::mutex> l(m_);
        cv_.wait(l, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        if (w >= nt_) continue;
        job = job_;
      }
      (*job)(w);
      {
        std::lock_guard<std::mutex> l(m_);
        if (--left_ == 0) done_.notify_one();
      }
    }
  }
  int nw_;
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  std::function<void(int)>* job_ = nullptr;
  int nt_ = 0, left_ = 0;
  int64_t gen_ = 0;
  bool stop_ = false;
};

// Host wall-clock accumulators for the verbose report.
struct HostTimers {
  double t[16] = {0};
  Clock::time_point last = Clock::now();
  void mark(int i) {
    auto now = Clock::now();
    t[i] += std::chrono::duration<double>(now - last).count();
    last = now;
  }
};

// One worker thread for host jobs that nothing waits on until the end of the factorization
// (grouping the solve records' scatter lists); it runs while the planning thread waits on
// the device. Jobs run in submission order; drain() returns once all have finished and
// rethrows the first exception one of them raised.
class Background {
 public:
  Background() : th_([this] { loop(); }) {}
  ~Background() {
    {
      std::lock_guard<std::mutex> l(m_);
      stop_ = true;
    }
    cv_.notify_all();
    th_.join();
  }
  void post(std::function<void()> job) {
    {
      std::lock_guard<std::mutex> l(m_);
      q_.push_back(std::move(job));
      ++posted_;
    }
    cv_.notify_all();
  }
  void drain() {
    std::unique_lock<std::mutex> l(m_);
    idle_.wait(l, [&] { return done_ == posted_; });
    if (err_) {
      std::exception_ptr e = err_;
      err_ = nullptr;
      std::rethrow_exception(e);
    }
  }

 private:
  void loop() {
    for (;;) {
      std::function<void()> job;
      {
        std::unique_lock<std::mutex> l(m_);
        cv_.wait(l, [&] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;  // stop requested and nothing left
        job = std::move(q_.front());
        q_.pop_front();
      }
      std::exception_ptr e;
      try {
        job();
      } catch (...) {
        e = std::current_exception();
      }
      {
        std::lock_guard<std::mutex> l(m_);
        if (e && !err_) err_ = e;
        ++done_;
      }
      idle_.notify_all();
    }
  }
  std::mutex m_;
  std::condition_variable cv_, idle_;
  std::deque<std::function<void()>> q_;
  int64_t posted_ = 0, done_ = 0;
  bool stop_ = false;
  std::exception_ptr err_;
  std::thread th_;
};

// Two scratch buffers used alternately by consecutive colour phases: the rank read-back of
// phase p waits for everything queued before phase p's ID, which includes all of phase
// p-1's work, so the buffer of phase p-1 can be recycled by phase p+1 without a wait.
class DoubleArena {
 public:
  void* alloc(size_t b) { return a_[cur_].alloc(b); }
  template <class T>
  T* alloc_n(size_t n) {
    return a_[cur_].alloc_n<T>(n);
  }
  void reset() { a_[cur_].reset(); }
  void reset_all() {
    a_[0].reset();
    a_[1].reset();
  }
  void flip() {
    cur_ ^= 1;
    a_[cur_].reset();
  }

 private:
  DeviceArena a_[2] = {DeviceArena(size_t(512) << 20), DeviceArena(size_t(512) << 20)};
  int cur_ = 0;

 public:
  // chunks from the factorization's device memory; the owner (Stage) drains its stream before
  // the arenas go
  void attach(DeviceMemory* m) {
    a_[0].set_memory(m);
    a_[1].set_memory(m);
  }
};
class DoubleHostStage {
 public:
  void* alloc(size_t b) { return h_[cur_].alloc(b); }
  void reset() { h_[cur_].reset(); }
  void reset_all() {
    h_[0].reset();
    h_[1].reset();
  }
  void flip() {
    cur_ ^= 1;
    h_[cur_].reset();
  }

 private:
  HostStage h_[2];
  int cur_ = 0;
};

// Upload chunks (pinned host memory and its device twin) outlive the factorization that
// allocated them: later factorizations of the process take them back instead of pinning new
// host memory (about a millisecond per few tens of megabytes). At most kChunkCacheMax bytes
// are kept; the cache is never torn down (the process exit reclaims it).
struct UploadChunk {
  void* h;
  void* d;
  size_t cap;
  int dev;
};
class ChunkCache {
 public:
  static constexpr size_t kChunkCacheMax = size_t(512) << 20;
  static ChunkCache& get() {
    static ChunkCache* c = new ChunkCache;  // not destroyed: no HIP calls at static teardown
    return *c;
  }
  // smallest cached chunk of this device holding at least b bytes
  bool take(size_t b, int dev, UploadChunk& out) {
    std::lock_guard<std::mutex> l(m_);
    int best = -1;
    for (int i = 0; i < (int)free_.size(); ++i)
      if (free_[i].dev == dev && free_[i].cap >= b && (best < 0 || free_[i].cap < free_[best].cap)) best = i;
    if (best < 0) return false;
    out = free_[best];
    held_ -= out.cap;
    free_.erase(free_.begin() + best);
    return true;
  }
  void trim() {
    std::vector<UploadChunk> all;
    {
      std::lock_guard<std::mutex> l(m_);
      all.swap(free_);
      held_ = 0;
    }
    for (auto& c : all) {
      (void)hipHostFree(c.h);
      (void)hipFree(c.d);
    }
  }
  void give(const UploadChunk& c) {
    {
      std::lock_guard<std::mutex> l(m_);
      if (held_ + c.cap <= kChunkCacheMax) {
        free_.push_back(c);
        held_ += c.cap;
        return;
      }
    }
    (void)hipHostFree(c.h);
    (void)hipFree(c.d);
  }

 private:
  std::mutex m_;
  std::vector<UploadChunk> free_;
  size_t held_ = 0;
};

// Task descriptors on their way to the device: pinned host and device buffers of equal size,
// bump-allocated at the same offsets, so the uploads queued between two launches leave in
// one copy. Chunks are kept for reuse; reset() only after the device is done with them.
class UploadRing {
 public:
  // the owner drains the stream before the ring goes, so no copy still reads a chunk
  ~UploadRing() {
    for (auto& c : chunks_) {
      if (mem_ && mem_->caller_allocator()) {
        (void)hipHostFree(c.h);
        mem_->put(c.d, c.cap);
      } else {
        if (mem_) mem_->unaccount(c.cap);
        ChunkCache::get().give(c);
      }
    }
  }
  // device memory the chunks are counted in (and, with a caller allocator, allocated from)
  void attach(DeviceMemory* m) { mem_ = m; }
  bool pending() const { return cur_ < chunks_.size() && flushed_ < used_; }
  // host and device addresses of b bytes (the caller flushes first when told to)
  bool fits(size_t b) const { return cur_ < chunks_.size() && used_ + align(b) <= chunks_[cur_].cap; }
  std::pair<void*, void*> alloc(size_t b) {
    b = align(b);
    if (!fits(b)) {
      // next chunk that fits, else a new one (pending bytes of the current chunk are
      // flushed by the caller before this point)
      size_t next = cur_ < chunks_.size() ? cur_ + 1 : 0;
      while (next < chunks_.size() && chunks_[next].cap < b) ++next;
      if (next >= chunks_.size()) {
        UploadChunk c{};
        int dev = 0;
        FMMLU_HIP(hipGetDevice(&dev));
        if (mem_ && mem_->caller_allocator()) {
          c.cap = std::max(b, size_t(16) << 20);
          c.dev = dev;
          FMMLU_HIP(hipHostMalloc(&c.h, c.cap, hipHostMallocDefault));
          try {
            c.d = mem_->get(c.cap, c.cap);
          } catch (...) {
            (void)hipHostFree(c.h);
            throw;
          }
        } else {
          if (!ChunkCache::get().take(b, dev, c)) {
            c.cap = std::max(b, size_t(16) << 20);
            c.dev = dev;
            FMMLU_HIP(hipHostMalloc(&c.h, c.cap, hipHostMallocDefault));
            if (hipMalloc(&c.d, c.cap) != hipSuccess) {
              (void)hipGetLastError();
              (void)hipHostFree(c.h);
              throw Error(FMMLU_ENOMEM, "upload buffer allocation failed");
            }
          }
          if (mem_) {
            try {
              mem_->account(c.cap);
            } catch (...) {
              ChunkCache::get().give(c);
              throw;
            }
          }
        }
        chunks_.push_back(c);
        next = chunks_.size() - 1;
      }
      cur_ = next;
      used_ = flushed_ = 0;
    }
    UploadChunk& c = chunks_[cur_];
    std::pair<void*, void*> r{static_cast<char*>(c.h) + used_, static_cast<char*>(c.d) + used_};
    used_ += b;
    return r;
  }
  void flush(hipStream_t st) {
    if (!pending()) return;
    UploadChunk& c = chunks_[cur_];
    FMMLU_HIP(hipMemcpyAsync(static_cast<char*>(c.d) + flushed_, static_cast<char*>(c.h) + flushed_,
                             used_ - flushed_, hipMemcpyHostToDevice, st));
    flushed_ = used_;
  }
  void reset() {
    cur_ = 0;
    used_ = flushed_ = 0;
  }

 private:
  static size_t align(size_t b) { return std::max<size_t>((b + 255) & ~size_t(255), 256); }
  DeviceMemory* mem_ = nullptr;
  std::vector<UploadChunk> chunks_;
  size_t cur_ = 0, used_ = 0, flushed_ = 0;
};

struct Stage {
  // device scratch and pinned staging, double-buffered across colour phases
  DoubleArena dev;
  DoubleHostStage host;
  UploadRing ring[2];
  int rcur = 0;
  hipStream_t st = nullptr;
  Profiler* prof = nullptr;
  // scratch and upload buffers counted in (and taken from) a factorization's device memory
  void attach(DeviceMemory* m) {
    dev.attach(m);
    ring[0].attach(m);
    ring[1].attach(m);
  }
  // the buffers are freed only once the stream's work on them has finished (also when an
  // error unwinds the factorization); members are destroyed after this body runs
  ~Stage() {
    if (st) (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
  }
  // a point in the stream that the host can wait for without waiting for what follows it
  hipEvent_t ev = nullptr;
  void mark() {
    flush();
    if (!ev) FMMLU_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    FMMLU_HIP(hipEventRecord(ev, st));
  }
  void wait_mark() {
    auto a = std::chrono::steady_clock::now();
    FMMLU_HIP(hipEventSynchronize(ev));
    t_wait += std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  }
  // switch to the other buffer at the start of a colour phase (see DoubleArena)
  void flip() {
    flush();
    dev.flip();
    host.flip();
    rcur ^= 1;
    ring[rcur].reset();
  }
  // queued uploads leave in one copy; every launch that may read them goes through go()
  void flush() { ring[rcur].flush(st); }
  hipStream_t go() {
    flush();
    return st;
  }

  template <class T>
  T* up(const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    const size_t b = v.size() * sizeof(T);
    UploadRing& r = ring[rcur];
    if (!r.fits(b)) r.flush(st);
    auto hd = r.alloc(b);
    std::memcpy(hd.first, v.data(), b);
    return static_cast<T*>(hd.second);
  }
  // upload space for n values that the caller fills in place on the host (before the next
  // go()): the host and device addresses
  template <class T>
  std::pair<T*, T*> up_raw(size_t n) {
    if (n == 0) return {nullptr, nullptr};
    const size_t b = n * sizeof(T);
    UploadRing& r = ring[rcur];
    if (!r.fits(b)) r.flush(st);
    auto hd = r.alloc(b);
    return {static_cast<T*>(hd.first), static_cast<T*>(hd.second)};
  }
  // persistent upload into another arena
  template <class T>
  T* up_to(DeviceArena& a, const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    size_t b = v.size() * sizeof(T);
    void* h = host.alloc(b);
    std::memcpy(h, v.data(), b);
    T* d = static_cast<T*>(a.alloc(b));
    FMMLU_HIP(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, st));
    return d;
  }
  // several persistent uploads in one device allocation and one copy: add() records where
  // each array's device address goes, commit() allocates, stages and copies them all
  struct Packed {
    struct Part {
      const void* src;
      size_t bytes, off;
      void** out;
    };
    std::vector<Part> parts;
    size_t total = 0;
    template <class T>
    void add(T** out, const std::vector<T>& v) {
      *out = nullptr;
      if (v.empty()) return;
      total = (total + 255) & ~size_t(255);
      parts.push_back(Part{v.data(), v.size() * sizeof(T), total, reinterpret_cast<void**>(out)});
      total += v.size() * sizeof(T);
    }
  };
  void commit(DeviceArena& a, Packed& pk) {
    if (pk.parts.empty()) return;
    char* h = static_cast<char*>(host.alloc(pk.total));
    char* d = static_cast<char*>(a.alloc(pk.total));
    for (auto& p : pk.parts) {
      std::memcpy(h + p.off, p.src, p.bytes);
      *p.out = d + p.off;
    }
    FMMLU_HIP(hipMemcpyAsync(d, h, pk.total, hipMemcpyHostToDevice, st));
    pk.parts.clear();
    pk.total = 0;
  }
  double t_wait = 0;
  void sync() {
    flush();
    auto a = std::chrono::steady_clock::now();
    FMMLU_HIP(hipStreamSynchronize(st));
    t_wait += std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  }
  void sync_reset() {
    sync();
    if (prof) prof->harvest();
    dev.reset_all();
    host.reset_all();
    ring[0].reset();
    ring[1].reset();
  }
};

// Units of a GEMM task: kGemmTile x kGemmTile output blocks
inline int64_t gemm_units(int M, int N) {
  return int64_t((M + kGemmTile - 1) / kGemmTile) * ((N + kGemmTile - 1) / kGemmTile);
}
inline int64_t units64(int r, int c) { return int64_t((r + 63) / 64) * ((c + 63) / 64); }

constexpr int64_t kUnitMapMax = int64_t(1) << 22;  // largest grid given a block -> task map

struct GemmBatch {
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
  int64_t units = 0;
  void add(void* C, int ldc, int M, int N, const int32_t* rmap, const int32_t* cmap,
           const std::vector<GemmSeg>& s, double are, double aim, double beta, bool lower = false) {
    if (M <= 0 || N <= 0) return;
    GemmTask t{};
    t.lower = lower && M == N ? 1 : 0;
    t.C = C;
    t.rmap = rmap;
    t.cmap = cmap;
    t.M = M;
    t.N = N;
    t.ldc = ldc;
    t.seg_begin = (int32_t)segs.size();
    t.nseg = (int32_t)s.size();
    t.alpha_re = are;
    t.alpha_im = aim;
    t.beta = beta;
    t.unit_begin = units;
    units += gemm_task_tiles(M, N, t.lower);
    for (auto& g : s) segs.push_back(g);
    tasks.push_back(t);
  }
  // C_part[k] = alpha * A^op B over K chunk k (k < ceil(K / kchunk)); partials at stride pstride.
  // lower (M == N): only the output tiles on or below the diagonal are formed.
  void add_split(zd* Cpart, int ldc, int M, int N, const zd* A, int lda, const zd* B, int ldb, int K,
                 int kchunk, int64_t pstride, bool lower = false) {
    if (M <= 0 || N <= 0 || K <= 0) return;
    const int nsplit = (K + kchunk - 1) / kchunk;
    GemmTask t{};
    t.C = Cpart;
    t.M = M;
    t.N = N;
    t.ldc = ldc;
    t.seg_begin = (int32_t)segs.size();
    t.nseg = 1;
    t.kchunk = kchunk;
    t.lower = lower && M == N ? 1 : 0;
    t.part_stride = pstride;
    t.alpha_re = 1.0;
    t.beta = 0.0;
    t.unit_begin = units;
    units += gemm_task_tiles(M, N, t.lower) * nsplit;
    segs.push_back(GemmSeg{A, B, lda, ldb, K, 0});
    tasks.push_back(t);
  }
  void add1(void* C, int ldc, int M, int N, const zd* A, int lda, const zd* B, int ldb, int K,
            double are, double beta) {
    if (K <= 0) {
      if (beta == 1.0) return;
    }
    std::vector<GemmSeg> s;
    if (K > 0) s.push_back(GemmSeg{A, B, lda, ldb, K, 0});
    add(C, ldc, M, N, nullptr, nullptr, s, are, 0.0, beta);
  }
  GemmTask* dt = nullptr;
  GemmSeg* ds = nullptr;
  int32_t* du = nullptr;  // task of each output block (one read per workgroup on the device)
  void prepare(Stage& sg) {
    if (tasks.empty()) return;
    dt = sg.up(tasks);
    ds = sg.up(segs);
    du = nullptr;
    // the map needs one batch-wide prefix (batches concatenated from separate launches
    // restart it and keep the search)
    const int nt = (int)tasks.size();
    bool one_prefix = units > 0 && units <= kUnitMapMax && tasks[0].unit_begin == 0;
    for (int i = 1; i < nt && one_prefix; ++i) one_prefix = tasks[i].unit_begin >= tasks[i - 1].unit_begin;
    if (one_prefix && tasks[nt - 1].unit_begin <= units) {
      std::vector<int32_t> ut((size_t)units);
      for (int i = 0; i < nt; ++i) {
        const int64_t e = i + 1 < nt ? tasks[i + 1].unit_begin : units;
        std::fill(ut.begin() + tasks[i].unit_begin, ut.begin() + e, (int32_t)i);
      }
      du = sg.up(ut);
    }
  }
  void launch(Stage& sg, int opA, bool c32 = false) {
    if (tasks.empty()) return;
    bool mapped = false;
    int64_t kmax = 0;  // longest inner dimension of one product (the autotuner's bucket)
    for (auto& t : tasks) {
      mapped = mapped || t.rmap || t.cmap;
      int64_t k = 0;
      for (int q = 0; q < t.nseg; ++q) k += segs[(size_t)t.seg_begin + q].K;
      kmax = std::max<int64_t>(kmax, t.kchunk > 0 ? std::min<int64_t>(k, t.kchunk) : k);
    }
    launch_gemm(opA, dt, (int)tasks.size(), units, ds, c32, sg.go(), mapped, du,
                gemm_tuned_kernel(c32, mapped, opA, kmax));
  }
  void run(Stage& sg, int opA) {
    prepare(sg);
    launch(sg, opA);
  }
};

// Batched Gauss-Jordan inversion of matrices A_b (n_b x n_b, lda_b) into out_b (ld n_b).
// All descriptors are uploaded first; the launches are timed as class `cls`.
void batched_inverse_pipeline(Stage& sg, std::vector<GjTask>& tasks, const std::vector<zd*>& outs,
                              int32_t* info_dev, int cls) {
  if (tasks.empty()) return;
  int nmax = 0;
  for (auto& t : tasks) nmax = std::max(nmax, t.n);
  const int nt = (int)tasks.size();
  std::vector<zd*> W(nt);
  std::vector<int32_t*> work(nt);
  // panel groups: single-workgroup matrices in one launch; taller ones cooperatively, in
  // groups whose grid (count x widest) fits the device
  int nmulti = 0;
  for (auto& t : tasks) nmulti += gj_wpt(t.n) > 1 ? 1 : 0;
  int32_t* counters = nmulti ? sg.dev.alloc_n<int32_t>(nmulti) : nullptr;
  if (nmulti) FMMLU_HIP(hipMemsetAsync(counters, 0, sizeof(int32_t) * nmulti, sg.go()));
  int ci = 0;
  for (int i = 0; i < nt; ++i) {
    GjTask& t = tasks[i];
    t.piv = sg.dev.alloc_n<int32_t>(t.n);
    t.info = info_dev;
    t.wpt = gj_wpt(t.n);
    t.slots = nullptr;
    t.counter = nullptr;
    if (t.wpt > 1) {
      t.slots = sg.dev.alloc_n<zd>((size_t)(2 * gj_slot_len(t.wpt)));
      t.counter = counters + ci++;
    }
    W[i] = sg.dev.alloc_n<zd>((size_t)kGjBlock * t.n);
    work[i] = sg.dev.alloc_n<int32_t>(t.n);
  }
  GjTask* dt = sg.up(tasks);
  struct PanelGroup {
    GjTask* dt;
    int count, wmax;
  };
  std::vector<PanelGroup> pgroups;
  {
    std::vector<GjTask> single, multi;
    for (auto& t : tasks) (t.wpt > 1 ? multi : single).push_back(t);
    if (!single.empty()) pgroups.push_back({sg.up(single), (int)single.size(), 1});
    if (!multi.empty()) {
      std::stable_sort(multi.begin(), multi.end(), [](const GjTask& a, const GjTask& b) { return a.wpt < b.wpt; });
      const int cap = gj_panel_capacity();
      size_t b = 0;
      while (b < multi.size()) {
        size_t e = b;
        int wmax = 0;
        while (e < multi.size() && (int64_t)(e - b + 1) * std::max(wmax, multi[e].wpt) <= cap) {
          wmax = std::max(wmax, multi[e].wpt);
          ++e;
        }
        if (e == b) throw Error(FMMLU_EINVAL, "pivot block too large for one cooperative panel launch");
        std::vector<GjTask> grp(multi.begin() + (int64_t)b, multi.begin() + (int64_t)e);
        pgroups.push_back({sg.up(grp), (int)grp.size(), wmax});
        b = e;
      }
    }
  }
  zd** dW = sg.up(W);
  int32_t** dwork = sg.up(work);
  zd** dout = sg.up(outs);
  // all steps' GEMM descriptors are concatenated into one batch and uploaded once
  GemmBatch all;
  std::vector<std::array<int64_t, 4>> sidx;  // task begin, count, unit base, units
  for (int j0 = 0; j0 < nmax; j0 += kGjBlock) {
    GemmBatch gb;
    for (int i = 0; i < nt; ++i) {
      const GjTask& t = tasks[i];
      if (j0 >= t.n) continue;
      const int nb = std::min(kGjBlock, t.n - j0);
      // A[:, c] += A[:, J] W[:, c] for c outside J (two column ranges)
      // A[:, c] += (A[:, J] - E_J) W[:, c] for c outside J (E_J: identity on rows J), which
      // also subtracts the pivot rows W from rows J
      const GemmSeg seg{t.A + (int64_t)j0 * t.lda, nullptr, t.lda, nb, nb, j0 + 1};
      if (j0 > 0) {
        GemmSeg g = seg;
        g.B = W[i];
        gb.add(t.A, t.lda, t.n, j0, nullptr, nullptr, {g}, 1.0, 0.0, 1.0);
      }
      const int c1 = j0 + nb;
      if (c1 < t.n) {
        GemmSeg g = seg;
        g.B = W[i] + (int64_t)c1 * nb;
        gb.add(t.A + (int64_t)c1 * t.lda, t.lda, t.n, t.n - c1, nullptr, nullptr, {g}, 1.0, 0.0, 1.0);
      }
    }
    const int64_t tb = (int64_t)all.tasks.size();
    const int64_t seg0 = (int64_t)all.segs.size();
    for (auto t : gb.tasks) {
      t.seg_begin += (int32_t)seg0;
      all.tasks.push_back(t);
    }
    for (auto& g : gb.segs) all.segs.push_back(g);
    sidx.push_back({tb, (int64_t)gb.tasks.size(), 0, gb.units});
  }
  all.prepare(sg);
  ProfScope ps(*sg.prof, cls);
  int step = 0;
  for (int j0 = 0; j0 < nmax; j0 += kGjBlock, ++step) {
    for (auto& pg : pgroups) launch_gj_panel(pg.dt, pg.count, j0, pg.wmax, sg.go());
    launch_gj_swapcopy(dt, nt, j0, nmax, dW, sg.go());
    if (sidx[step][1] > 0)
      launch_gemm(0, all.dt + sidx[step][0], (int)sidx[step][1], sidx[step][3], all.ds, false, sg.go());
  }
  launch_gj_unpermute(dt, nt, nmax, dout, dwork, sg.go());
  for (auto& t : tasks) sg.prof->flops[cls] += 8.0 * (double)t.n * t.n * t.n;
}

// Inverses of a batch of matrices: those up to kGjCoopMax rows in cooperative launches
// (several workgroups per matrix, one launch for the whole inversion), larger ones through
// the multi-launch pipeline.
void batched_inverse(Stage& sg, std::vector<GjTask>& tasks, const std::vector<zd*>& outs, int32_t* info_dev,
                     int cls) {
  std::vector<GjTask> large;
  std::vector<zd*> lo;
  std::vector<GjCoopTask> small;
  for (size_t i = 0; i < tasks.size(); ++i) {
    if (tasks[i].n <= kGjCoopMax) {
      GjCoopTask c{};
      c.A = tasks[i].A;
      c.out = outs[i];
      c.n = tasks[i].n;
      c.lda = tasks[i].lda;
      small.push_back(c);
    } else {
      large.push_back(tasks[i]);
      lo.push_back(outs[i]);
    }
  }
  if (!small.empty()) {
    int nmax = 0;
    for (auto& c : small) nmax = std::max(nmax, c.n);
    const int NB = gj_coop_panel(nmax);
    // per matrix: 2 npan + 1 synchronisation words of the cooperative kernel, zeroed
    size_t nsync = 0;
    for (auto& c : small) nsync += (size_t)gj_coop_sync_words(c.n, NB);
    int32_t* counters = sg.dev.alloc_n<int32_t>(nsync);
    FMMLU_HIP(hipMemsetAsync(counters, 0, sizeof(int32_t) * nsync, sg.go()));
    size_t so = 0;
    for (size_t i = 0; i < small.size(); ++i) {
      small[i].piv = sg.dev.alloc_n<int32_t>(small[i].n);
      small[i].info = info_dev;
      small[i].counter = counters + so;
      so += (size_t)gj_coop_sync_words(small[i].n, NB);
    }
    const int cap = gj_coop_capacity(nmax);
    // Workgroups per matrix: one per panel up to K, with K the largest that keeps the whole
    // batch at one workgroup per compute unit (a matrix's time is its panel chain; fewer
    // workgroups add each one's share of the column updates to that chain, and workgroups
    // sharing a compute unit slow each other's redundant panel work).
    // While other factorizations run concurrently, one workgroup per matrix: the launch then
    // has no waits between workgroups and goes out as an ordinary launch, where cooperative
    // launches would have to be serialised across the concurrent factorizations.
    auto npan_of = [NB](int n) { return (n + NB - 1) / NB; };
    const int64_t budget = std::min(cap, gj_coop_cus());
    int K = 1;
    for (int k = 2; ActiveFactorization::count() <= 1 && k <= npan_of(nmax); ++k) {
      int64_t tot = 0;
      for (auto& c : small) tot += std::min(npan_of(c.n), k);
      if (tot > budget) break;
      K = k;
    }
    for (auto& c : small) c.nwg = std::min(npan_of(c.n), K);
    size_t b = 0;
    while (b < small.size()) {
      std::vector<GjCoopTask> grp;
      int64_t units = 0;
      while (b < small.size() && units + small[b].nwg <= cap) {
        small[b].unit_begin = units;
        units += small[b].nwg;
        grp.push_back(small[b++]);
      }
      if (grp.empty()) throw Error(FMMLU_EINVAL, "pivot block too large for one cooperative launch");
      GjCoopTask* dt = sg.up(grp);
      ProfScope ps(*sg.prof, cls);
      launch_gj_coop(dt, (int)grp.size(), units, nmax, sg.go());
    }
    for (auto& t : small) sg.prof->flops[cls] += 8.0 * (double)t.n * t.n * t.n;
  }
  // up to kGjStepMax rows: one launch per panel; beyond, the blocked multi-launch pipeline
  std::vector<GjTask> huge;
  std::vector<zd*> ho;
  for (size_t i = 0; i < large.size(); ++i) {
    GjTask& t = large[i];
    if (t.n > kGjStepMax) {
      huge.push_back(t);
      ho.push_back(lo[i]);
      continue;
    }
    GjStepArgs a{};
    a.A = t.A;
    a.n = t.n;
    a.lda = t.lda;
    a.info = info_dev;
    a.piv = sg.dev.alloc_n<int32_t>(t.n);
    a.rowcol = sg.dev.alloc_n<int32_t>(t.n);
    FMMLU_HIP(hipMemsetAsync(a.rowcol, 0xFF, sizeof(int32_t) * t.n, sg.go()));  // all -1
    ProfScope ps(*sg.prof, cls);
    const int npan = (t.n + kGjStepNb - 1) / kGjStepNb;
    for (int j = -1; j < npan; ++j) launch_gj_step(a, j, sg.go());
    launch_gj_step_gather(a, lo[i], sg.go());
    sg.prof->flops[cls] += 8.0 * (double)t.n * t.n * t.n;
  }
  batched_inverse_pipeline(sg, huge, ho, info_dev, cls);
}

// Blocked Householder QR (no pivoting) of M_b (rows_b x m_b, ld rows_b), in place; the R
// factor is left in the upper triangle. Per panel of kQrBlock columns: panel kernel, then the
// trailing update A2 -= V (Tw^H (V^H A2)) with V^H A2 as a split-K GEMM (long K = panel height).
void batched_qr(Stage& sg, const std::vector<zd*>& Ms, const std::vector<int>& rows,
                const std::vector<int>& ms) {
  const int nt = (int)Ms.size();
  if (nt == 0) return;
  constexpr int NB = kQrBlock;
  constexpr int KCH = 512;
  int kmax = 0;
  for (int i = 0; i < nt; ++i) kmax = std::max(kmax, std::min(rows[i], ms[i]));
  std::vector<zd*> V(nt), Tw(nt), W2(nt), part(nt);
  for (int i = 0; i < nt; ++i) {
    V[i] = sg.dev.alloc_n<zd>((size_t)rows[i] * NB);
    Tw[i] = sg.dev.alloc_n<zd>(NB * NB);
    W2[i] = sg.dev.alloc_n<zd>((size_t)NB * ms[i]);
    const int nsplit = (rows[i] + KCH - 1) / KCH;
    part[i] = sg.dev.alloc_n<zd>((size_t)nsplit * NB * ms[i]);
  }
  struct Step {
    QrTask* dqt;
    int nq;
    GemmBatch g1, g3;
    RedTwTask* drt;
    int nrt, cmax;
  };
  std::vector<Step> steps;
  for (int j0 = 0; j0 < kmax; j0 += NB) {
    std::vector<QrTask> qt;
    std::vector<int> who;
    for (int i = 0; i < nt; ++i) {
      const int k = std::min(rows[i], ms[i]);
      if (j0 >= k) continue;
      QrTask t{};
      t.A = Ms[i];
      t.V = V[i];
      t.Tw = Tw[i];
      t.rows = rows[i];
      t.lda = rows[i];
      t.j0 = j0;
      t.nb = std::min(NB, k - j0);
      qt.push_back(t);
      who.push_back(i);
    }
    if (qt.empty()) break;
    Step stp;
    stp.dqt = sg.up(qt);
    stp.nq = (int)qt.size();
    std::vector<RedTwTask> rt;
    stp.cmax = 0;
    for (size_t q = 0; q < qt.size(); ++q) {
      const int i = who[q];
      const int nb = qt[q].nb;
      const int c0 = j0 + nb;
      const int ncols = ms[i] - c0;
      if (ncols <= 0) continue;
      const int L = rows[i] - j0;
      zd* A2 = Ms[i] + j0 + (int64_t)c0 * rows[i];
      const int64_t pstride = (int64_t)nb * ncols;
      stp.g1.add_split(part[i], nb, nb, ncols, V[i], L, A2, rows[i], L, KCH, pstride);
      rt.push_back(RedTwTask{part[i], Tw[i], W2[i], nb, ncols, (L + KCH - 1) / KCH, 0, pstride});
      stp.cmax = std::max(stp.cmax, ncols);
      stp.g3.add1(A2, rows[i], L, ncols, V[i], L, W2[i], nb, nb, -1.0, 1.0);
    }
    stp.g1.prepare(sg);
    stp.g3.prepare(sg);
    stp.drt = sg.up(rt);
    stp.nrt = (int)rt.size();
    steps.push_back(std::move(stp));
  }
  {
    ProfScope ps(*sg.prof, KC_QR);
    for (auto& stp : steps) {
      launch_qr_panel(stp.dqt, stp.nq, sg.go());
      stp.g1.launch(sg, 2);
      if (stp.nrt) launch_reduce_tw(stp.drt, stp.nrt, stp.cmax, sg.go());
      stp.g3.launch(sg, 0);
    }
  }
  for (int i = 0; i < nt; ++i) {
    const double L = rows[i], m = std::min(rows[i], ms[i]), n = ms[i];
    // complex Householder QR of an L x n matrix: ~ L n^2 - n^3/3 complex MACs
    sg.prof->flops[KC_QR] += 8.0 * (L * n * m - m * m * m / 3.0);
  }
}

}  // namespace

void trim_reuse_caches() {
  ChunkCache::get().trim();
  PinnedCache::get().trim();
  DeviceChunkCache::get().trim();
}

// Inverses of count consecutive n x n matrices (the routine the factorization uses for the
// pivot blocks and the top block), for the library's dense-inverse entry point.
void dense_inverse_batch(const zd* A, int64_t n, int64_t count, zd* out, hipStream_t st) {
  Profiler prof;
  Stage sg;
  sg.st = st;
  sg.prof = &prof;
  DeviceArena keep(size_t(1) << 20);
  int32_t* info_dev = keep.alloc_n<int32_t>(1);
  FMMLU_HIP(hipMemsetAsync(info_dev, 0, sizeof(int32_t), st));
  zd* work = keep.alloc_n<zd>((size_t)(n * n * count));
  FMMLU_HIP(hipMemcpyAsync(work, A, sizeof(zd) * (size_t)(n * n * count), hipMemcpyDeviceToDevice, st));
  std::vector<GjTask> tasks((size_t)count);
  std::vector<zd*> outs((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    tasks[i] = GjTask{};
    tasks[i].A = work + i * n * n;
    tasks[i].n = (int32_t)n;
    tasks[i].lda = (int32_t)n;
    outs[i] = out + i * n * n;
  }
  batched_inverse(sg, tasks, outs, info_dev, KC_INV);
  int32_t hinfo = 0;
  FMMLU_HIP(hipMemcpyAsync(&hinfo, info_dev, sizeof(int32_t), hipMemcpyDeviceToHost, sg.go()));
  sg.sync_reset();
  if (hinfo < 0) throw Error(FMMLU_EHIP, "Gauss-Jordan panel barrier timed out");
  if (hinfo != 0) throw Error(FMMLU_ESINGULAR, "zero pivot in column " + std::to_string(hinfo - 1));
}


// A colour phase's solve record before its scatter lists are grouped and uploaded (done at
// the end of the factorization, overlapping the top block on the device).
struct PendingPhase {
  SolvePhase ph;
  std::vector<std::pair<int32_t, int64_t>> contrib;  // (destination, y index)
  std::vector<SolveBox> db;
  std::vector<SweepTask> txr, ty, tbp, tbt, tbt16;
  std::vector<SweepTask> txr16, ty16, tbp16;  // single-vector items of 16 outputs / rows
  std::vector<SweepTask> txs;                 // blocked: backward x_R sums, 64 entries of R
  std::vector<int32_t> dst;
  std::vector<int64_t> ptr, src;
};

// Owner geometry for the pair search: level and cell coordinates at that level.
struct OwnerCell {
  int level;
  int64_t c[3];
};

// Close lists of a set of disjoint owner boxes: for each owner (ascending, unique) the owners
// covering the cells within two of its own at its level, plus every finer owner that found
// it (a coarser owner cannot find a finer one back). At the finest depth D each owner
// covers the Morton key range [klo, khi); the owner containing a cell of level lev is the
// one whose range holds the cell's first key, if that owner's level is <= lev. Runs on the
// pool's threads when one is given.
std::vector<std::vector<int>> close_owner_lists(const std::vector<OwnerCell>& ow, int D, HostPool* hp) {
  const int no = (int)ow.size();
  std::vector<uint64_t> klo(no), khi(no);
  std::vector<int> kown(no);
  for (int i = 0; i < no; ++i) {
    const int sh = D - ow[i].level;
    klo[i] = morton3((uint32_t)(ow[i].c[0] << sh), (uint32_t)(ow[i].c[1] << sh), (uint32_t)(ow[i].c[2] << sh));
    khi[i] = klo[i] + (uint64_t(1) << (3 * sh));
    kown[i] = i;
  }
  std::sort(kown.begin(), kown.end(), [&](int a, int b) { return klo[a] < klo[b]; });
  auto lookup = [&](int lev, int64_t x, int64_t y, int64_t z) -> int {
    const int64_t lim = int64_t(1) << lev;
    if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return -1;
    const int sh = D - lev;
    const uint64_t key = morton3((uint32_t)(x << sh), (uint32_t)(y << sh), (uint32_t)(z << sh));
    auto it = std::upper_bound(kown.begin(), kown.end(), key, [&](uint64_t k, int o) { return k < klo[o]; });
    if (it == kown.begin()) return -1;
    const int o = *(it - 1);
    return (key < khi[o] && ow[o].level <= lev) ? o : -1;
  };
  std::vector<std::vector<int>> close(no);
  auto search = [&](int lo, int hi) {
    for (int i = lo; i < hi; ++i) {
      const OwnerCell& o = ow[i];
      auto& v = close[i];
      for (int dz = -2; dz <= 2; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
          for (int dx = -2; dx <= 2; ++dx) {
            const int p = lookup(o.level, o.c[0] + dx, o.c[1] + dy, o.c[2] + dz);
            if (p >= 0) v.push_back(p);
          }
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
  };
  if (hp)
    hp->ranges(no, 64, search);
  else
    search(0, no);
  std::vector<std::vector<int>> back(no);
  for (int i = 0; i < no; ++i)
    for (int p : close[i])
      if (ow[p].level < ow[i].level) back[p].push_back(i);
  for (int p = 0; p < no; ++p) {
    if (back[p].empty()) continue;
    auto& v = close[p];
    v.insert(v.end(), back[p].begin(), back[p].end());
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  return close;
}

// The close pairs that get a tile (gap of at most one box), owner by owner in ascending
// order: beg (per owner, CSR), ids (the partner), pairs ((owner, partner) in that order).
void tile_pairs(const std::vector<OwnerCell>& ow, const std::vector<std::vector<int>>& close,
                std::vector<int64_t>& beg, std::vector<int32_t>& ids, std::vector<std::pair<int, int>>& pairs) {
  const int no = (int)ow.size();
  beg.assign(1, 0);
  ids.clear();
  pairs.clear();
  for (int i = 0; i < no; ++i) {
    for (int p : close[i]) {
      if (gap_units(ow[i], ow[p]) > 1) continue;
      ids.push_back(p);
      pairs.emplace_back(i, p);
    }
    beg.push_back((int64_t)ids.size());
  }
}

// Scatter lists of a phase grouped by destination (CSR): y indices increase with the box
// order, so sorting the (destination, y) pairs keeps each destination's contributions in box
// order. The pair list is released afterwards.
void group_scatter(PendingPhase& pp) {
  auto& contrib = pp.contrib;
  std::sort(contrib.begin(), contrib.end());
  pp.ptr.assign(1, 0);
  pp.dst.reserve(contrib.size());
  pp.src.reserve(contrib.size());
  for (size_t k = 0; k < contrib.size(); ++k) {
    if (k > 0 && contrib[k].first != contrib[k - 1].first) pp.ptr.push_back((int64_t)pp.src.size());
    if (k == 0 || contrib[k].first != contrib[k - 1].first) pp.dst.push_back(contrib[k].first);
    pp.src.push_back(contrib[k].second);
  }
  if (!contrib.empty()) pp.ptr.push_back((int64_t)pp.src.size());
  std::vector<std::pair<int32_t, int64_t>>().swap(contrib);
}

// ------------------------------------------------------------------------------------------
void FactorImpl::factor(const Octree& tree, const double* xyz, const double* nrm, const double* w,
                        hipStream_t st) {
  const ActiveFactorization active;
  auto t0 = Clock::now();
  n = tree.n;
  f32 = opts.precision == FMMLU_FP32;
  const size_t te = f32 ? sizeof(zf) : sizeof(zd);  // bytes per stored tile or factor entry
  info = fmmlu_info{};
  info.n = n;
  info.nlevels = tree.nlevels;
  info.precision = opts.precision;
  mem.configure(opts, st);
  // measure the GEMM kernels on this device once per process (later calls return at once);
  // 2, 3, 4 force one kernel for every GEMM of this factorization (testing)
  struct ForceReset {
    ~ForceReset() { gemm_force_kernel(GK_AUTO); }
  } force_reset;
  if (opts.gemm_autotune == 1) gemm_autotune(mem, st);
  gemm_force_kernel(opts.gemm_autotune >= 2 ? opts.gemm_autotune - 2 : GK_AUTO);
  // whatever is released after this call (also when an error unwinds it) is ordered on the
  // null stream: the caller's stream may be gone by then
  struct StreamReset {
    DeviceMemory& m;
    ~StreamReset() { m.set_stream(nullptr); }
  } stream_reset{mem};
  arena.set_memory(&mem);  // freed by the destructor after the device has drained
  rarena.set_memory(&mem);
  farena.set_memory(&mem);
  Stage sg;
  sg.st = st;
  sg.attach(&mem);
  HostPool hp((int)std::min(8u, std::max(1u, std::thread::hardware_concurrency())));
  prof.on = opts.profile != 0;
  prof.mask = opts.profile == 2 ? (1u << KC_SCHUR) : ~0u;
  prof.st = st;
  sg.prof = &prof;
  // ---- geometry in tree order: x, y, z, nx, ny, nz, sqrt(w)
  order = tree.order;
  {
    std::vector<double> gp(7 * (size_t)n);
    for (int64_t p = 0; p < n; ++p) {
      const int64_t o = order[p];
      for (int a = 0; a < 3; ++a) {
        gp[a * n + p] = xyz[a * n + o];
        gp[(3 + a) * n + p] = nrm[a * n + o];
      }
      gp[6 * n + p] = std::sqrt(w[o]);
    }
    geom = sg.up_to(arena, gp);
    order_dev = sg.up_to(arena, order);
  }
  g = DevGeom{geom, n, k, eta};
  if (n > 0) {
    // k times the bounding box's diagonal bounds the phase k r of every pair of points
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double lo = xyz[a * n], hi = lo;
      for (int64_t p = 1; p < n; ++p) {
        lo = std::min(lo, xyz[a * n + p]);
        hi = std::max(hi, xyz[a * n + p]);
      }
      d2 += (hi - lo) * (hi - lo);
    }
    g.kr_max = k * std::sqrt(d2) * (1.0 + 1e-12);
  }
  // ---- quadrature corrections (Section 5.3): tree-order CSR by row and by column on the
  // device; on the host, every position's partners (either direction) for the spill-over rule
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
  if (opts.corr_row_ptr) {
    std::vector<int64_t> pos(n);
    for (int64_t p = 0; p < n; ++p) pos[order[p]] = p;
    // tree-order CSR by row and by column: counts, offsets, one scatter, then every segment
    // sorted on the host workers; a position's partners merge its two sorted segments
    std::vector<int64_t> rptr(n + 1, 0), cptr(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = opts.corr_row_ptr[i]; e < opts.corr_row_ptr[i + 1]; ++e) {
        const int64_t j = opts.corr_col[e];
        if (j == i) continue;  // the diagonal is 1/2, not a quadrature entry
        ++rptr[pos[i] + 1];
        ++cptr[pos[j] + 1];
      }
    for (int64_t p = 0; p < n; ++p) {
      rptr[p + 1] += rptr[p];
      cptr[p + 1] += cptr[p];
    }
    const int64_t nnz = rptr[n];
    std::vector<std::pair<int32_t, double>> rv((size_t)nnz), cv((size_t)nnz);
    {
      std::vector<int64_t> rf(rptr.begin(), rptr.end() - 1), cf(cptr.begin(), cptr.end() - 1);
      for (int64_t i = 0; i < n; ++i) {
        const int64_t pi = pos[i];
        for (int64_t e = opts.corr_row_ptr[i]; e < opts.corr_row_ptr[i + 1]; ++e) {
          const int64_t j = opts.corr_col[e];
          if (j == i) continue;
          const int64_t pj = pos[j];
          rv[(size_t)rf[pi]++] = {(int32_t)pj, opts.corr_a[e]};
          cv[(size_t)cf[pj]++] = {(int32_t)pi, opts.corr_a[e]};
        }
      }
    }
    std::vector<int32_t> rcol((size_t)nnz), crow((size_t)nnz);
    std::vector<double> ra((size_t)nnz), ca((size_t)nnz);
    adj_ptr.assign(n + 1, 0);
    std::atomic<bool> twice{false};
    // position p's partners in either direction, ascending without repeats (counted only
    // when out is null)
    auto partners = [&](int64_t p, int32_t* out) {
      auto r = rv.cbegin() + rptr[p], re = rv.cbegin() + rptr[p + 1];
      auto c = cv.cbegin() + cptr[p], ce = cv.cbegin() + cptr[p + 1];
      int64_t k = 0;
      int32_t last = -1;
      while (r != re || c != ce) {
        const int32_t v = (c == ce || (r != re && r->first <= c->first)) ? (r++)->first : (c++)->first;
        if (k == 0 || v != last) {
          if (out) out[k] = v;
          ++k;
          last = v;
        }
      }
      return k;
    };
    hp.ranges((int)n, 512, [&](int lo, int hi) {
      for (int64_t p = lo; p < hi; ++p) {
        const auto rb = rv.begin() + rptr[p], re = rv.begin() + rptr[p + 1];
        const auto cb = cv.begin() + cptr[p], ce = cv.begin() + cptr[p + 1];
        std::sort(rb, re);
        std::sort(cb, ce);
        for (auto it = rb; it != re; ++it) {
          if (it != rb && it->first == (it - 1)->first) twice = true;
          rcol[(size_t)(it - rv.begin())] = it->first;
          ra[(size_t)(it - rv.begin())] = it->second;
        }
        for (auto it = cb; it != ce; ++it) {
          crow[(size_t)(it - cv.begin())] = it->first;
          ca[(size_t)(it - cv.begin())] = it->second;
        }
        adj_ptr[p + 1] = partners(p, nullptr);
      }
    });
    if (twice) throw Error(FMMLU_EINVAL, "correction table lists a pair twice");
    for (int64_t p = 0; p < n; ++p) adj_ptr[p + 1] += adj_ptr[p];
    adj.resize((size_t)adj_ptr[n]);
    hp.ranges((int)n, 512, [&](int lo, int hi) {
      for (int64_t p = lo; p < hi; ++p) partners(p, adj.data() + adj_ptr[p]);
    });
    g.corr.rptr = sg.up_to(arena, rptr);
    g.corr.rcol = sg.up_to(arena, rcol);
    g.corr.ra = sg.up_to(arena, ra);
    g.corr.cptr = sg.up_to(arena, cptr);
    g.corr.crow = sg.up_to(arena, crow);
    g.corr.ca = sg.up_to(arena, ca);
  }
  // the caller's table is only valid during this call: nothing keeps its pointers
  opts.corr_row_ptr = nullptr;
  opts.corr_col = nullptr;
  opts.corr_a = nullptr;
  std::vector<uint8_t> pos_live(adj_ptr.empty() ? 0 : (size_t)n, 1);  // active at the phase start
  const double eps = opts.eps;
  const double prad = opts.proxy_radius;

  // ---- initial owners: every non-empty leaf, points in tree order (contiguous)
  std::vector<Owner> own;
  for (int b = 0; b < (int)tree.nboxes(); ++b) {
    if (!tree.is_leaf(b) || tree.npts(b) == 0) continue;
    Owner o;
    o.box = b;
    o.level = tree.level[b];
    o.c[0] = tree.cx[b];
    o.c[1] = tree.cy[b];
    o.c[2] = tree.cz[b];
    o.first_pos = tree.first_pos(b);
    o.act.resize(tree.npts(b));
    std::iota(o.act.begin(), o.act.end(), o.first_pos);
    own.push_back(std::move(o));
  }
  std::sort(own.begin(), own.end(), [](const Owner& a, const Owner& b) { return a.first_pos < b.first_pos; });
  int64_t live_total = n;

  // tiles of the previous level (for assembly). Two pools used alternately by consecutive
  // levels and grown on demand. A pool outgrown at a level boundary may still be read by work
  // queued on st: it is retired and freed after the next rank read-back, which has waited for
  // that work anyway (a free is not ordered with the stream, and another thread's allocation
  // could reuse the memory).
  void* prev_pool = nullptr;
  void* pools[2] = {nullptr, nullptr};
  size_t pool_cap[2] = {0, 0};
  int pool_slot = 0;
  std::vector<std::pair<void*, size_t>> retired;
  struct PoolGuard {
    void** p;
    std::vector<std::pair<void*, size_t>>* r;
    hipStream_t st;
    size_t* cap;
    DeviceMemory* mem;
    ~PoolGuard() {
      (void)hipStreamSynchronize(st);
      for (int i = 0; i < 2; ++i)
        if (p[i]) mem->put(p[i], cap[i]);
      for (auto& q : *r) mem->put(q.first, q.second);
    }
  } pool_guard{pools, &retired, st, pool_cap, &mem};
  // per-level device lists stay alive until the factorization has drained
  std::vector<std::unique_ptr<DeviceArena>> level_arenas;
  std::deque<PendingPhase> pending;  // solve records (stable addresses for the grouping jobs)
  Background bgw;                     // declared after pending: its jobs end before pending goes
  // destroyed first: no buffer above is freed while kernels queued on st may still use it
  struct DrainOnExit {
    hipStream_t st;
    ~DrainOnExit() { (void)hipStreamSynchronize(st); }
  } drain_on_exit{st};
  PairIndex prev_pidx;  // pairs of the previous level's owners
  std::vector<Owner> prev_own;
  bool first_level = true;
  int32_t* info_dev = arena.alloc_n<int32_t>(1);
  FMMLU_HIP(hipMemsetAsync(info_dev, 0, sizeof(int32_t), st));

  const int D = std::max(tree.nlevels - 1, 0);
  // close lists of the next level's owners, computed ahead on a worker thread (see below);
  // the worker is declared last so that its job ends before the lists it writes go
  std::vector<int> spec_boxes;
  struct SpecLevel {
    std::vector<std::vector<int>> close;
    std::vector<int64_t> beg;
    std::vector<int32_t> ids;
    std::vector<std::pair<int, int>> pairs;
  } spec;
  bool spec_posted = false;
  Background spec_worker;

  HostTimers ht;
  // largest rank seen at this level and at the level before (bounds for the blocked pivoting)
  int rank_max_level = 0, rank_max_prev = 0;
  int pchol_continued = 0;  // phases whose blocked pivoting ran past the bound (verbose report)
  for (int lev = tree.nlevels - 1; lev >= 2; --lev) {
    const int nown = (int)own.size();
    if (rank_max_level > 0) rank_max_prev = rank_max_level;
    rank_max_level = 0;
    // ---- close pairs of owners and their tiles: taken from the worker's speculative lists
    // when this level's owners are the ones it assumed, else searched here
    std::vector<std::vector<int>> close;
    PairIndex pidx;
    std::vector<std::pair<int, int>> pairs;
    bool spec_hit = false;
    if (spec_posted) {
      spec_worker.drain();
      spec_posted = false;
      bool same = (int)spec_boxes.size() == nown;
      for (int i = 0; same && i < nown; ++i) same = spec_boxes[i] == own[i].box;
      if (same) {
        close.swap(spec.close);
        pidx.beg.swap(spec.beg);
        pidx.ids.swap(spec.ids);
        pairs.swap(spec.pairs);
      }
      spec_hit = same;
      spec = SpecLevel{};
    }
    if (!spec_hit) {
      std::vector<OwnerCell> cells(nown);
      for (int i = 0; i < nown; ++i) cells[i] = OwnerCell{own[i].level, {own[i].c[0], own[i].c[1], own[i].c[2]}};
      close = close_owner_lists(cells, D, &hp);
      tile_pairs(cells, close, pidx.beg, pidx.ids, pairs);
    }
    // the next level's owners if every owner keeps live DOFs (the merge below checks): the
    // parents of this level's boxes and the coarser owners, in tree order; their close
    // lists depend on geometry only
    if (lev - 1 >= 2) {
      std::vector<std::pair<int64_t, int>> nb;  // (a tree position inside the box, box)
      std::unordered_map<int, int> seen;
      for (const Owner& o : own) {
        const int tb = o.level == lev ? tree.parent[o.box] : o.box;
        if (seen.emplace(tb, 1).second) nb.emplace_back(o.first_pos, tb);
      }
      std::sort(nb.begin(), nb.end());
      spec_boxes.resize(nb.size());
      std::vector<OwnerCell> cells(nb.size());
      for (size_t i = 0; i < nb.size(); ++i) {
        const int b = nb[i].second;
        spec_boxes[i] = b;
        cells[i] = OwnerCell{(int)tree.level[b], {(int64_t)tree.cx[b], (int64_t)tree.cy[b], (int64_t)tree.cz[b]}};
      }
      spec_worker.post([&spec, cells = std::move(cells), D] {
        spec.close = close_owner_lists(cells, D, nullptr);
        tile_pairs(cells, spec.close, spec.beg, spec.ids, spec.pairs);
      });
      spec_posted = true;
    }
    // tile offsets in the level's pool (pair order)
    std::vector<int32_t> kcount;  // per pair, zero between colour phases (Schur grouping)
    int64_t pool_elems = 0;
    pidx.off.resize(pairs.size());
    for (size_t k = 0; k < pairs.size(); ++k) {
      pidx.off[k] = pool_elems;
      pool_elems += (int64_t)own[pairs[k].first].act.size() * own[pairs[k].second].act.size();
    }
    kcount.assign(pidx.ids.size(), 0);
    ht.mark(0);
    void* pool = nullptr;
    {
      const size_t bytes = std::max<size_t>(1, (size_t)pool_elems) * te;
      const int ps = pool_slot;
      pool_slot ^= 1;
      if (pool_cap[ps] < bytes) {
        // the previous level's assembly, still queued on st, may be reading this pool
        if (pools[ps]) retired.emplace_back(pools[ps], pool_cap[ps]);
        pools[ps] = nullptr;
        pool_cap[ps] = 0;
        size_t got = bytes;
        void* pp = mem.get(bytes, got);
        pools[ps] = pp;
        pool_cap[ps] = got;
      }
      pool = pools[ps];
    }
    info.bytes_tiles += (double)pool_elems * (double)te;
    ht.mark(8);
    // ---- assemble: slot/idx maps, dof lists, source tables
    {
      std::vector<int32_t> slot, idx;
      std::vector<int64_t> dof;
      std::vector<int64_t> map_off(nown);
      for (int i = 0; i < nown; ++i) {
        Owner& o = own[i];
        map_off[i] = (int64_t)slot.size();
        if (first_level) {
          for (size_t r = 0; r < o.act.size(); ++r) {
            slot.push_back(0);
            idx.push_back((int32_t)r);
          }
        } else {
          for (size_t q = 0; q < o.sub.size(); ++q) {
            const Owner& so = prev_own[o.sub[q]];
            for (int32_t l : so.live) {
              slot.push_back((int32_t)q);
              idx.push_back(l);
            }
          }
        }
        for (int64_t a : o.act) dof.push_back(a);
      }
      // tasks and source tables of all pairs: sizes first, then filled on host threads
      const int np = (int)pairs.size();
      std::vector<int64_t> tabo(np + 1, 0), unito(np + 1, 0);
      for (int k = 0; k < np; ++k) {
        const Owner& a = own[pairs[k].first];
        const Owner& b = own[pairs[k].second];
        tabo[k + 1] = tabo[k] + (first_level ? 1 : (int64_t)a.sub.size() * (int64_t)b.sub.size());
        const bool live = !a.act.empty() && !b.act.empty();
        unito[k + 1] = unito[k] + (live ? units64((int)a.act.size(), (int)b.act.size()) : 0);
      }
      // the source table is written straight into its upload space (no copy)
      const std::pair<AsmSrc*, AsmSrc*> table = sg.up_raw<AsmSrc>((size_t)tabo[np]);
      std::vector<AsmTask> all((size_t)np);
      hp.ranges(np, 256, [&](int lo, int hi) {
        for (int k = lo; k < hi; ++k) {
          const auto& pr = pairs[k];
          const Owner& a = own[pr.first];
          const Owner& b = own[pr.second];
          AsmTask t{};
          t.out_off = pidx.off[k];
          t.nr = (int)a.act.size();
          t.nc = (int)b.act.size();
          t.ld = t.nr;
          t.rmap_off = map_off[pr.first];
          t.cmap_off = map_off[pr.second];
          t.rdof_off = map_off[pr.first];
          t.cdof_off = map_off[pr.second];
          t.tab_off = tabo[k];
          AsmSrc* tab = table.first + tabo[k];
          if (first_level) {
            t.nsc = 1;
            tab[0] = AsmSrc{-1, 0, 0};
          } else {
            t.nsc = (int)b.sub.size();
            int64_t e = 0;
            for (int sa : a.sub)
              for (int sb : b.sub) {
                const int64_t o = prev_pidx.find(sa, sb);
                tab[e++] = o < 0 ? AsmSrc{-1, 0, 0} : AsmSrc{o, (int32_t)prev_own[sa].act.size(), 0};
              }
          }
          t.unit_begin = unito[k];
          all[k] = t;
        }
      });
      std::vector<AsmTask> tasks;
      tasks.reserve(all.size());
      for (auto& t : all)
        if (t.nr > 0 && t.nc > 0) tasks.push_back(t);
      const int64_t units = unito[np];
      // task of each 64 x 64 unit (one read per workgroup in place of a search)
      std::vector<int32_t> ut;
      if (units <= kUnitMapMax) {
        ut.resize((size_t)units);
        const int ntk = (int)tasks.size();
        for (int k = 0; k < ntk; ++k) {
          const int64_t e = k + 1 < ntk ? tasks[k + 1].unit_begin : units;
          std::fill(ut.begin() + tasks[k].unit_begin, ut.begin() + e, (int32_t)k);
        }
      }
      {
        AsmTask* dt = sg.up(tasks);
        int32_t* dslot = sg.up(slot);
        int32_t* didx = sg.up(idx);
        int64_t* ddof = sg.up(dof);
        AsmSrc* dtab = table.second;
        int32_t* dut = sg.up(ut);
        ProfScope ps(prof, KC_ASSEMBLE);
        launch_assemble(g, dt, (int)tasks.size(), units, dslot, didx, ddof, dtab, prev_pool, f32, pool, f32, sg.go(),
                        dut);
      }
      prof.bytes[KC_ASSEMBLE] += (double)te * (double)pool_elems * (first_level ? 1.0 : 2.0);
      prev_pool = nullptr;
    }
    // every owner starts the level fully live; device copies of act positions as int32 tree
    // positions are kept per owner for the factor records
    for (auto& o : own) {
      o.live.resize(o.act.size());
      std::iota(o.live.begin(), o.live.end(), 0);
    }
    // device live lists: identity for all owners at level start
    {
      std::vector<int32_t> ident;
      int maxc = 0;
      for (auto& o : own) maxc = std::max<int>(maxc, (int)o.act.size());
      ident.resize(maxc);
      std::iota(ident.begin(), ident.end(), 0);
      int32_t* dident = sg.up_to(arena, ident);  // persistent for the level (small)
      for (auto& o : own) o.live_dev = dident;
    }
    // device copy of all act lists (int64 tree positions) for the ID matrix proxy rows
    std::vector<int64_t> act_cat;
    std::vector<int64_t> act_off(nown);
    for (int i = 0; i < nown; ++i) {
      act_off[i] = (int64_t)act_cat.size();
      act_cat.insert(act_cat.end(), own[i].act.begin(), own[i].act.end());
    }
    level_arenas.emplace_back(new DeviceArena(size_t(4) << 20, &mem));
    DeviceArena& level_arena = *level_arenas.back();
    int64_t* act_dev = sg.up_to(level_arena, act_cat);
    // owner of every position active at this level (spill-over rule)
    std::vector<int32_t> owner_of;
    // spill-over candidates of each owner processed at this level: (owner q, position p) for
    // every partner p of one of its positions whose owner q lies beyond the stored pairs
    // (gap of two units or more). Owners, their positions and their boxes stay fixed through
    // the level; whether p is still active is decided when the owner's phase is planned.
    std::vector<std::vector<std::pair<int, int32_t>>> spill_cand;
    if (!adj_ptr.empty()) {
      owner_of.assign((size_t)n, -1);
      for (int i = 0; i < nown; ++i)
        for (int64_t a : own[i].act) owner_of[(size_t)a] = i;
      spill_cand.assign((size_t)nown, {});
      hp.ranges(nown, 16, [&](int lo, int hi) {
        for (int i = lo; i < hi; ++i) {
          const Owner& B = own[i];
          if (B.level != lev) continue;
          auto& out = spill_cand[(size_t)i];
          for (int64_t a : B.act)
            for (int64_t e = adj_ptr[a]; e < adj_ptr[a + 1]; ++e) {
              const int32_t p = adj[e];
              const int q = owner_of[p];
              if (q < 0 || q == i) continue;
              if (gap_units(B, own[q]) >= 2) out.emplace_back(q, p);
            }
        }
      });
    }

    // ---- processed boxes by colour, Morton order within a colour
    std::vector<std::vector<int>> colours(8);
    for (int i = 0; i < nown; ++i) {
      const Owner& o = own[i];
      if (o.level != lev) continue;
      const int col = int(o.c[0] & 1) + 2 * int(o.c[1] & 1) + 4 * int(o.c[2] & 1);
      colours[col].push_back(i);
    }
    for (auto& v : colours)
      std::sort(v.begin(), v.end(), [&](int a, int b) {
        return morton3((uint32_t)own[a].c[0], (uint32_t)own[a].c[1], (uint32_t)own[a].c[2]) <
               morton3((uint32_t)own[b].c[0], (uint32_t)own[b].c[1], (uint32_t)own[b].c[2]);
      });

    ht.mark(1);
    for (int colour = 0; colour < 8; ++colour) {
      // ---- plan the phase
      struct BoxPlan {
        int oi;
        int m;
        std::vector<int> nown_, qown;  // near and Q owners (with live DOFs)
        std::vector<int> qspill;       // Q owners beyond the stored pairs (spill-over)
        int nN = 0, nQ = 0;
        bool far_p = false;
        int ngamma = 0;
        double ctr[3], radius = 0, wgamma = 0;
        int rows = 0;
        zd* M = nullptr;
        zd* R = nullptr;
        int32_t* perm = nullptr;
        int32_t* rank = nullptr;
        zd* T = nullptr;
      };
      std::vector<BoxPlan> plan;
      for (int oi : colours[colour]) {
        Owner& B = own[oi];
        if (B.live.empty()) continue;
        BoxPlan bp;
        bp.oi = oi;
        bp.m = (int)B.act.size();
        int64_t near_live = 0;
        for (int p : close[oi]) {
          if (p == oi) continue;
          const int64_t gu = gap_units(B, own[p]);
          if (own[p].live.empty()) continue;
          if (gu == 0) {
            bp.nown_.push_back(p);
            bp.nN += (int)own[p].live.size();
          } else if (gu == 1) {
            bp.qown.push_back(p);
            bp.nQ += (int)own[p].live.size();
          }
        }
        // Section 5.3: an owner beyond the stored pairs (in B's P region) linked to B by a
        // quadrature correction joins Q; its rows are generated (corrected kernel values)
        if (!adj_ptr.empty()) {
          std::vector<int> sp;
          for (const auto& cq : spill_cand[(size_t)oi])
            if (pos_live[(size_t)cq.second]) sp.push_back(cq.first);
          std::sort(sp.begin(), sp.end());
          sp.erase(std::unique(sp.begin(), sp.end()), sp.end());
          for (int q : sp) {
            bp.qown.push_back(q);
            bp.qspill.push_back(q);
            bp.nQ += (int)own[q].live.size();
          }
          info.nspill += (int32_t)sp.size();
        }
        near_live = (int64_t)bp.nN + bp.nQ + (int64_t)B.live.size();
        bp.far_p = live_total - near_live > 0;
        if (bp.nQ == 0 && !bp.far_p) continue;
        // owners are already in tree order (index order == first_pos order)
        std::sort(bp.nown_.begin(), bp.nown_.end());
        std::sort(bp.qown.begin(), bp.qown.end());
        const double side = tree.box_side(B.box);
        tree.box_centre(B.box, bp.ctr);
        if (bp.far_p) {
          const double ratio = prad / (std::sqrt(3.0) / 2.0);
          const int p = (int)std::ceil(std::log(1.0 / eps) / std::log(ratio)) +
                        (int)std::ceil(k * std::sqrt(3.0) * side);
          bp.ngamma = std::max(opts.proxy_min_points, 2 * (p + 1) * (p + 1));
          bp.radius = prad * side;
          bp.wgamma = std::sqrt(4.0 * M_PI * bp.radius * bp.radius / bp.ngamma);
        }
        bp.rows = 2 * bp.nQ + 2 * bp.ngamma;
        plan.push_back(std::move(bp));
      }
      if (plan.empty()) continue;
      // Only phases with work flip: each of them waits on its rank read-back below, which
      // is what makes the buffer of the phase before last free for reuse.
      sg.flip();
      const int nb = (int)plan.size();
      // Schur contributions of the plan's boxes (box q = plan entry q), each assumed to keep a
      // skeleton: contributions grouped by destination tile (tiles in pair order, boxes in
      // order within a tile); ok = false if a needed tile is not stored
      struct Contrib {
        int64_t toff;
        int64_t k;     // destination pair index (tiles lie in the pool in pair order)
        int q;         // box index
        int32_t a, b;  // group indices (0 = the box itself, else near owner index + 1)
      };
      struct SchurGroups {
        std::vector<std::vector<int>> grps;  // per box: its owner, then its near owners
        std::vector<Contrib> cl;             // grouped by destination tile
        std::vector<int32_t> first{0};       // tile u has cl[first[u], first[u + 1])
        bool ok = true;
      };
      auto schur_groups = [&](int nq) {
        SchurGroups G;
        G.grps.resize(nq);
        std::vector<std::vector<Contrib>> pcl(nq);  // per box, built on host threads
        std::vector<int> bad(nq, 0);
        hp.ranges(nq, 4, [&](int lo, int hi) {
          for (int q = lo; q < hi; ++q) {
            const BoxPlan& bp = plan[q];
            auto& grp = G.grps[q];
            grp.push_back(bp.oi);
            for (int o : bp.nown_) grp.push_back(o);
            for (size_t a = 0; a < grp.size(); ++a)
              for (size_t b = 0; b < grp.size(); ++b) {
                const int M = (a == 0) ? 1 : (int)own[grp[a]].live.size();
                const int N = (b == 0) ? 1 : (int)own[grp[b]].live.size();
                if (M == 0 || N == 0) continue;
                const int64_t k = pidx.pos(grp[a], grp[b]);
                if (k < 0) {
                  bad[q] = 1;
                  continue;
                }
                pcl[q].push_back(Contrib{pidx.off[k], k, q, (int32_t)a, (int32_t)b});
              }
          }
        });
        for (int q = 0; q < nq; ++q)
          if (bad[q]) G.ok = false;
        // group by destination tile, boxes in order within a tile: count per touched pair
        // (kcount is all zero between uses), order the touched pairs, place stably
        std::vector<int64_t> tk;
        size_t ncl = 0;
        for (auto& v : pcl) {
          ncl += v.size();
          for (auto& c : v)
            if (kcount[c.k]++ == 0) tk.push_back(c.k);
        }
        std::sort(tk.begin(), tk.end());
        const int ntk = (int)tk.size();
        G.first.assign(ntk + 1, 0);
        for (int u = 0; u < ntk; ++u) {
          G.first[u + 1] = G.first[u] + kcount[tk[u]];
          kcount[tk[u]] = G.first[u];  // now the fill position of pair tk[u]
        }
        G.cl.resize(ncl);
        for (auto& v : pcl)
          for (auto& c : v) G.cl[kcount[c.k]++] = c;
        for (int u = 0; u < ntk; ++u) kcount[tk[u]] = 0;
        return G;
      };
      ht.mark(2);
      // ---- 1. ID matrices
      std::vector<IdTask> idt;
      std::vector<QSeg> qsegs;
      int64_t units = 0;
      for (auto& bp : plan) {
        Owner& B = own[bp.oi];
        bp.M = sg.dev.alloc_n<zd>((size_t)bp.rows * bp.m);
        IdTask t{};
        t.M = bp.M;
        t.rows = bp.rows;
        t.m = bp.m;
        t.nq = bp.nQ;
        t.ngamma = bp.ngamma;
        t.seg_off = (int64_t)qsegs.size();
        int row0 = 0;
        for (int q : bp.qown) {
          QSeg s{};
          if (std::binary_search(bp.qspill.begin(), bp.qspill.end(), q)) {
            s.tile_qb = s.tile_bq = -1;
            s.gdof = act_dev + act_off[q];
          } else {
            s.tile_qb = pidx.at(q, bp.oi);
            s.tile_bq = pidx.at(bp.oi, q);
          }
          s.live = own[q].live_dev;
          s.ld = (int)own[q].act.size();
          s.row0 = row0;
          row0 += (int)own[q].live.size();
          qsegs.push_back(s);
        }
        t.nseg = (int)bp.qown.size();
        t.dof_off = act_off[bp.oi];
        t.cx = bp.ctr[0];
        t.cy = bp.ctr[1];
        t.cz = bp.ctr[2];
        t.radius = bp.radius;
        t.wgamma = bp.wgamma;
        t.unit_begin = units;
        units += units64(t.rows, t.m);
        idt.push_back(t);
        (void)B;
      }
      {
        IdTask* didt = sg.up(idt);
        QSeg* dq = qsegs.empty() ? nullptr : sg.up(qsegs);
        ProfScope ps(prof, KC_IDMAT);
        launch_build_idmatrix(g, didt, nb, units, dq, act_dev, pool, f32, sg.go());
      }
      for (auto& bp : plan) prof.bytes[KC_IDMAT] += 16.0 * (double)bp.rows * bp.m;
      // ---- 2. greedy CPQR of M: through the Gram matrix (pivoted Cholesky of M^H M) when
      //      eps >= kGramEps, else Householder QR of M followed by CPQR of its R factor
      // ranks and pivots of all boxes of the phase in two contiguous arrays (one read-back each)
      int64_t perm_total = 0;
      for (auto& bp : plan) perm_total += bp.m;
      int32_t* rank_all = sg.dev.alloc_n<int32_t>(nb);
      int32_t* perm_all = sg.dev.alloc_n<int32_t>((size_t)perm_total);
      {
        int64_t po = 0;
        for (int i = 0; i < nb; ++i) {
          plan[i].rank = rank_all + i;
          plan[i].perm = perm_all + po;
          po += plan[i].m;
        }
      }
      int32_t* hr = nullptr;  // host copy of ranks and pivots (set where the read-back is queued)
      // blocked pivoted Cholesky: the blocks past the predicted bound (run only when a box's
      // pivoting had not stopped by then), and those blocks with a second read-back
      std::function<void()> pchol_more, pchol_rest;
      GemmBatch gu;  // the blocked pivoting's downdates of G (used by pchol_more as well)
      const bool gram = opts.id_route == 1 || (opts.id_route == 0 && eps >= kGramEps);
      if (gram) {
        constexpr int KCH = 512;
        GemmBatch gg;
        std::vector<SumTask> st_;
        std::vector<PcholTask> pt;
        int64_t su = 0;
        int mmax = 0;
        for (auto& bp : plan) {
          const int nsplit = (bp.rows + KCH - 1) / KCH;
          const int64_t mm = (int64_t)bp.m * bp.m;
          zd* part = sg.dev.alloc_n<zd>((size_t)nsplit * mm);
          zd* G = sg.dev.alloc_n<zd>((size_t)mm);
          bp.R = sg.dev.alloc_n<zd>((size_t)mm);
          bp.T = sg.dev.alloc_n<zd>((size_t)mm);
          // G = M^H M is Hermitian: its lower triangle of tiles, completed by the sum of the
          // split-K partials (the pivoting reads rows of G as contiguous columns)
          gg.add_split(part, bp.m, bp.m, bp.m, bp.M, bp.rows, bp.M, bp.rows, bp.rows, KCH, mm, true);
          SumTask sm{part, G, mm, mm, nsplit, bp.m, su};
          su += (mm + 255) / 256;
          st_.push_back(sm);
          zd* Rp = sg.dev.alloc_n<zd>((size_t)mm);
          pt.push_back(PcholTask{G, bp.R, Rp, bp.perm, bp.rank, bp.T, bp.m, 0, nullptr, nullptr, nullptr});
          mmax = std::max(mmax, bp.m);
          prof.flops[KC_QR] += 4.0 * (double)bp.rows * bp.m * (bp.m + 1);
        }
        // wide blocks: the blocked form (pivots in blocks of kPcholNb, G downdated between
        // blocks by a batched GEMM on all compute units) instead of one workgroup streaming
        // every earlier row of R at every pivot
        const bool blocked = mmax >= kPcholBlockedMin && mmax <= kPcholThreadsB;
        if (blocked) {
          for (size_t i = 0; i < plan.size(); ++i) {
            PcholTask& t = pt[i];
            const int m = t.m;
            t.Rb = sg.dev.alloc_n<zd>((size_t)kPcholNb * m);
            t.dgs = sg.dev.alloc_n<double>((size_t)m + 1);
            t.ist = sg.dev.alloc_n<int32_t>((size_t)2 * m + 2);
            gu.add(t.G, m, m, m, nullptr, nullptr, {GemmSeg{t.Rb, t.Rb, kPcholNb, kPcholNb, kPcholNb, 0}}, -1.0, 0.0,
                   1.0, false);
            gu.tasks.back().skip = t.ist + 2 * m + 1;  // no downdate once the box's pivoting stopped
          }
          gu.prepare(sg);
        }
        gg.prepare(sg);
        SumTask* dst_ = sg.up(st_);
        PcholTask* dpt = sg.up(pt);
        {
          ProfScope ps(prof, KC_QR);
          gg.launch(sg, 2);
          launch_sum_parts(dst_, (int)st_.size(), su, sg.go());
        }
        {
          ProfScope ps(prof, KC_CPQR);
          if (blocked) {
            // blocks up to a bound on the phase's ranks (from the ranks seen so far); a box
            // whose pivoting has not stopped there gets the remaining blocks after the rank
            // read-back (pchol_more): the same sequence of blocks either way
            const int nblk = (mmax + kPcholNb - 1) / kPcholNb;
            int bound = mmax;
            if (rank_max_level > 0)
              bound = (5 * rank_max_level) / 4 + kPcholNb;
            else if (rank_max_prev > 0)
              bound = (5 * rank_max_prev) / 2 + kPcholNb;
            int nb1 = std::min(nblk, bound / kPcholNb + 1);
            if (opts.pchol_blocks > 0) nb1 = std::min(nb1, opts.pchol_blocks);
            for (int b = 0; b < nb1; ++b) {
              launch_pchol_block(dpt, nb, b * kPcholNb, eps, sg.go(), mmax);
              if (b + 1 < nblk) gu.launch(sg, 2);
            }
            launch_pchol_finish(dpt, nb, mmax, sg.go());
            if (nb1 < nblk)
              pchol_more = [&, dpt, nb1, nblk, mmax, nb] {
                ProfScope ps2(prof, KC_CPQR);
                for (int b = nb1; b < nblk; ++b) {
                  launch_pchol_block(dpt, nb, b * kPcholNb, eps, sg.go(), mmax);
                  if (b + 1 < nblk) gu.launch(sg, 2);
                }
                launch_pchol_finish(dpt, nb, mmax, sg.go());
              };
          } else {
            launch_pchol(dpt, nb, mmax, eps, sg.go());
          }
        }
        // ranks and pivots are final here: their read-back goes ahead of T's back
        // substitution, which then runs while the host plans the elimination
        hr = static_cast<int32_t*>(sg.host.alloc(sizeof(int32_t) * (size_t)(nb + perm_total)));
        FMMLU_HIP(hipMemcpyAsync(hr, rank_all, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, sg.go()));
        FMMLU_HIP(hipMemcpyAsync(hr + nb, perm_all, sizeof(int32_t) * perm_total, hipMemcpyDeviceToHost, sg.go()));
        sg.mark();
        {
          ProfScope ps(prof, KC_CPQR);
          launch_pchol_t(dpt, nb, mmax, sg.go());
        }
        if (pchol_more)
          pchol_rest = [&, dpt, mmax, nb, perm_total, rank_all, perm_all] {
            pchol_more();
            FMMLU_HIP(hipMemcpyAsync(hr, rank_all, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, sg.go()));
            FMMLU_HIP(
                hipMemcpyAsync(hr + nb, perm_all, sizeof(int32_t) * perm_total, hipMemcpyDeviceToHost, sg.go()));
            sg.mark();
            {
              ProfScope ps(prof, KC_CPQR);
              launch_pchol_t(dpt, nb, mmax, sg.go());
            }
            sg.wait_mark();
          };
      } else {
        std::vector<zd*> Ms;
        std::vector<int> rws, mms;
        for (auto& bp : plan) {
          Ms.push_back(bp.M);
          rws.push_back(bp.rows);
          mms.push_back(bp.m);
        }
        batched_qr(sg, Ms, rws, mms);
        std::vector<ExtractTask> et;
        std::vector<CpqrTask> ct;
        int mmax = 0;
        for (auto& bp : plan) {
          bp.R = sg.dev.alloc_n<zd>((size_t)bp.m * bp.m);
          bp.T = sg.dev.alloc_n<zd>((size_t)bp.m * bp.m);
          et.push_back(ExtractTask{bp.M, bp.R, bp.rows, bp.m});
          zd* W = sg.dev.alloc_n<zd>((size_t)bp.m * bp.m / 4 + bp.m + 1);
          ct.push_back(CpqrTask{bp.R, bp.perm, bp.rank, bp.T, W, bp.m, bp.m});
          mmax = std::max(mmax, bp.m);
        }
        ExtractTask* det = sg.up(et);
        CpqrTask* dct = sg.up(ct);
        {
          ProfScope ps(prof, KC_CPQR);
          launch_extract_r(det, nb, mmax, sg.go());
          launch_cpqr(dct, nb, mmax, eps, sg.go());
        }
      }
      // ---- Schur structure of the phase, built while the device computes the IDs: for every
      //      box the destination tiles of its contributions (its own skeleton and near owners,
      //      pairwise), grouped by destination tile with boxes in order within a tile; after the
      //      read-back it is restricted to the boxes that eliminate something
      const SchurGroups sg_pre = schur_groups(nb);
      // ---- and the rank-independent parts of the elimination plan: per box its tile (B, B),
      //      the segments of its near owners and the N part of its S u N list (the near
      //      owners are of other colours: their live lists do not change in this phase)
      std::vector<int64_t> pre_tile_bb(nb);
      std::vector<std::vector<NSeg>> pre_nseg(nb);
      std::vector<std::vector<int32_t>> pre_nlist(nb);
      hp.ranges(nb, 8, [&](int lo, int hi) {
        for (int i = lo; i < hi; ++i) {
          const BoxPlan& bp = plan[i];
          pre_tile_bb[i] = pidx.find(bp.oi, bp.oi);
          auto& sgs = pre_nseg[i];
          auto& nl = pre_nlist[i];
          nl.reserve((size_t)bp.nN);
          int off = 0;
          for (int o : bp.nown_) {
            NSeg sgm{};
            sgm.tile_nb = pidx.find(o, bp.oi);
            sgm.tile_bn = pidx.find(bp.oi, o);
            sgm.live = own[o].live_dev;
            sgm.ld = (int)own[o].act.size();
            sgm.off = off;
            off += (int)own[o].live.size();
            sgs.push_back(sgm);
            for (int32_t l : own[o].live) nl.push_back((int32_t)own[o].act[l]);
          }
        }
      });
      // ---- read back ranks and pivots
      std::vector<int32_t> ranks(nb);
      std::vector<std::vector<int32_t>> perms(nb);
      {
        if (hr) {
          sg.wait_mark();
          bool open = false;
          for (int i = 0; i < nb; ++i) open = open || hr[i] < 0;
          if (open) {
            ++pchol_continued;
            if (!pchol_rest) throw Error(FMMLU_EINVAL, "internal: pivoting unfinished after every block");
            pchol_rest();
            for (int i = 0; i < nb; ++i)
              if (hr[i] < 0) throw Error(FMMLU_EINVAL, "internal: pivoting unfinished after every block");
          }
        } else {
          hr = static_cast<int32_t*>(sg.host.alloc(sizeof(int32_t) * (size_t)(nb + perm_total)));
          FMMLU_HIP(hipMemcpyAsync(hr, rank_all, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, sg.go()));
          FMMLU_HIP(hipMemcpyAsync(hr + nb, perm_all, sizeof(int32_t) * perm_total, hipMemcpyDeviceToHost, sg.go()));
          sg.sync();
        }
        for (auto& q : retired) mem.put(q.first, q.second);  // its readers have finished
        retired.clear();
        int64_t po = nb;
        for (int i = 0; i < nb; ++i) {
          ranks[i] = hr[i];
          perms[i].assign(hr + po, hr + po + plan[i].m);
          po += plan[i].m;
        }
      }
      for (int i = 0; i < nb; ++i) {
        double f = 0;
        for (int kk = 0; kk < ranks[i]; ++kk) f += 2.0 * (double)(plan[i].m - kk) * (plan[i].m - kk);
        prof.flops[KC_CPQR] += 8.0 * f;
        rank_max_level = std::max(rank_max_level, ranks[i]);
      }
      ht.mark(3);
      // ---- 3. elimination plan
      struct ElimPlan {
        int pi;  // index into plan
        int s, r, nsn;
        zd *Ccol, *Crow;
        zd* Up;  // X_RR^{-1} X_{R (S u N)} (r x nsn), scratch; stored transposed in the factor
        zd* Xi64;  // X_RR^{-1} in float64
        FactorBox* fb;
      };
      std::vector<ElimPlan> ep;
      const size_t box_base = boxes.size();
      for (int i = 0; i < nb; ++i) {
        const int s = ranks[i], m = plan[i].m;
        if (s >= m) continue;  // nothing redundant
        ElimPlan e{};
        e.pi = i;
        e.s = s;
        e.r = m - s;
        e.nsn = s + plan[i].nN;
        ep.push_back(e);
      }
      const int ne = (int)ep.size();
      if (ne > 0) {
        boxes.resize(box_base + ne);
        // factor storage and index lists
        std::vector<int32_t> idx_cat;
        std::vector<std::array<int64_t, 3>> idx_off(ne);
        int64_t idx_len = 0;
        std::vector<CrossTask> cross;
        std::vector<NSeg> nsegs;
        int64_t cunits = 0;
        for (int q = 0; q < ne; ++q) {
          ElimPlan& e = ep[q];
          BoxPlan& bp = plan[e.pi];
          Owner& B = own[bp.oi];
          FactorBox& fb = boxes[box_base + q];
          e.fb = &fb;
          fb.level = lev;
          fb.box = B.box;
          fb.coord[0] = (int)B.c[0];
          fb.coord[1] = (int)B.c[1];
          fb.coord[2] = (int)B.c[2];
          fb.m = bp.m;
          fb.s = e.s;
          fb.r = e.r;
          fb.nsn = e.nsn;
          // index lists of all boxes of the phase go up in one copy: R, S, then S u N (filled
          // on the host threads below)
          idx_off[q][0] = idx_len;
          idx_off[q][1] = idx_len + e.r;
          idx_off[q][2] = idx_len + e.r + e.s;
          idx_len += (int64_t)e.r + e.s + e.nsn;
          SolveBox& d = fb.dev;
          d.T = e.s ? arena.alloc(te * (size_t)e.s * e.r) : nullptr;
          d.Xi = arena.alloc(te * (size_t)e.r * e.r);
          d.Lp = e.nsn ? arena.alloc(te * (size_t)e.nsn * e.r) : nullptr;
          d.UpT = e.nsn ? arena.alloc(te * (size_t)e.r * e.nsn) : nullptr;
          // the inverse itself is formed in float64 (scratch when the factors are float32)
          e.Xi64 = f32 ? sg.dev.alloc_n<zd>((size_t)e.r * e.r) : static_cast<zd*>(const_cast<void*>(d.Xi));
          d.r = e.r;
          d.s = e.s;
          d.nsn = e.nsn;
          info.factor_bytes += (int64_t)te * ((int64_t)e.s * e.r + (int64_t)e.r * e.r + 2 * (int64_t)e.nsn * e.r);
          // cross gathers
          const int mn = bp.m + bp.nN;
          e.Ccol = sg.dev.alloc_n<zd>((size_t)mn * bp.m);
          e.Crow = sg.dev.alloc_n<zd>((size_t)bp.m * mn);
          CrossTask ct{};
          ct.Ccol = e.Ccol;
          ct.Crow = e.Crow;
          ct.tile_bb = pre_tile_bb[e.pi];
          ct.perm = bp.perm;
          ct.m = bp.m;
          ct.nN = bp.nN;
          ct.s = e.s;
          ct.seg_off = (int64_t)nsegs.size();
          for (const NSeg& sgm : pre_nseg[e.pi]) {
            if (sgm.tile_nb < 0 || sgm.tile_bn < 0 || ct.tile_bb < 0)
              throw Error(FMMLU_EINVAL, "internal: tile of a pair that is not close");
            nsegs.push_back(sgm);
          }
          ct.nseg = (int)bp.nown_.size();
          ct.unit_begin = cunits;
          cunits += units64(mn, bp.m) + units64(bp.m, mn);
          cross.push_back(ct);
          info.max_rank = std::max(info.max_rank, e.s);
        }
        idx_cat.resize((size_t)idx_len);
        std::vector<int> short_sn(ne, 0);
        hp.ranges(ne, 8, [&](int lo, int hi) {
          for (int q = lo; q < hi; ++q) {
            const ElimPlan& e = ep[q];
            const BoxPlan& bp = plan[e.pi];
            const Owner& B = own[bp.oi];
            const std::vector<int32_t>& pv = perms[e.pi];
            int32_t* rl = idx_cat.data() + idx_off[q][0];
            int32_t* sl = idx_cat.data() + idx_off[q][1];
            int32_t* sn = idx_cat.data() + idx_off[q][2];
            for (int j = 0; j < e.r; ++j) rl[j] = (int32_t)B.act[pv[e.s + j]];
            for (int j = 0; j < e.s; ++j) sl[j] = sn[j] = (int32_t)B.act[pv[j]];
            const std::vector<int32_t>& nl = pre_nlist[e.pi];
            if ((int64_t)e.s + (int64_t)nl.size() != e.nsn) {
              short_sn[q] = 1;
            } else if (!nl.empty()) {
              std::memcpy(sn + e.s, nl.data(), sizeof(int32_t) * nl.size());
            }
            FactorBox& fb = boxes[box_base + q];
            fb.skel_orig.resize(e.s);
            for (int j = 0; j < e.s; ++j) fb.skel_orig[j] = order[B.act[pv[j]]];
            std::sort(fb.skel_orig.begin(), fb.skel_orig.end());
          }
        });
        for (int q = 0; q < ne; ++q)
          if (short_sn[q]) throw Error(FMMLU_EINVAL, "internal: near-field list size changed within a phase");
        {
          int32_t* base = sg.up_to(arena, idx_cat);
          for (int q = 0; q < ne; ++q) {
            SolveBox& d = boxes[box_base + q].dev;
            d.R = base + idx_off[q][0];
            d.S = ep[q].s ? base + idx_off[q][1] : nullptr;
            d.SN = ep[q].nsn ? base + idx_off[q][2] : nullptr;
          }
        }
        ht.mark(9);
        CrossTask* dcross = sg.up(cross);
        NSeg* dns = nsegs.empty() ? nullptr : sg.up(nsegs);
        {
          ProfScope ps(prof, KC_ELIM);
          launch_gather_cross(dcross, ne, cunits, dns, pool, f32, sg.go());
        }
        ht.mark(10);
        // E/F transforms (Section 4.1). Ccol = A[(R,S,N),(S,R)], Crow = A[(S,R),(R,S,N)]:
        //   Ccol[:, s:m]      -= Ccol[:, 0:s] T        (A_{.R} - A_{.S} T)
        //   Ccol[0:r, s:m]    -= T^T Ccol[r:m, s:m]    -> X_RR;  Ccol[r:, s:m] = X_{(S u N) R}
        //   Crow[s:m, r:]     -= T^T Crow[0:s, r:]     -> X_{R (S u N)}
        {
          // ga first; gb depends on it. The Crow transform is independent of both and has
          // the same operand form as gb, so it goes in gb's launch.
          GemmBatch ga, gb;
          for (auto& e : ep) {
            BoxPlan& bp = plan[e.pi];
            const int m = bp.m, mn = bp.m + bp.nN;
            zd* CcR = e.Ccol + (int64_t)e.s * mn;
            ga.add1(CcR, mn, mn, e.r, e.Ccol, mn, bp.T, m, e.s, -1.0, 1.0);
            gb.add1(e.Crow + e.s + (int64_t)e.r * m, m, e.r, mn - e.r, bp.T, m, e.Crow + (int64_t)e.r * m, m,
                    e.s, -1.0, 1.0);
          }
          for (auto& e : ep) {
            BoxPlan& bp = plan[e.pi];
            const int m = bp.m, mn = bp.m + bp.nN;
            zd* CcR = e.Ccol + (int64_t)e.s * mn;
            gb.add1(CcR, mn, e.r, e.r, bp.T, m, CcR + e.r, mn, e.s, -1.0, 1.0);
            prof.flops[KC_ELIM] += 8.0 * ((double)mn * e.r * e.s + (double)e.r * (mn - e.r) * e.s +
                                          (double)e.r * e.r * e.s);
          }
          ga.prepare(sg);
          gb.prepare(sg);
          ProfScope ps(prof, KC_ELIM);
          ga.launch(sg, 0);
          gb.launch(sg, 1);
        }
        ht.mark(11);
        // 4. inverse of X_RR (in place in Ccol[0:r, 0:r]) -> Xi
        {
          std::vector<GjTask> gt;
          std::vector<zd*> outs;
          for (auto& e : ep) {
            GjTask t{};
            t.A = e.Ccol + (int64_t)e.s * (plan[e.pi].m + plan[e.pi].nN);
            t.n = e.r;
            t.lda = plan[e.pi].m + plan[e.pi].nN;
            gt.push_back(t);
            outs.push_back(e.Xi64);
            // failure-path testing: a pivot block forced to zero makes its inversion report
            // a zero pivot (FMMLU_ESINGULAR at the end of the factorization)
            if (opts.test_zero_pivot_block >= 0 && e.fb - boxes.data() == opts.test_zero_pivot_block)
              FMMLU_HIP(hipMemset2DAsync(t.A, sizeof(zd) * (size_t)t.lda, 0, sizeof(zd) * (size_t)t.n, (size_t)t.n,
                                         sg.go()));
          }
          batched_inverse(sg, gt, outs, info_dev, KC_INV);
        }
        ht.mark(12);
        // panels: Lp = X_{SN,R} Xi ; Up = Xi X_{R,SN}; T compacted into the factor
        {
          GemmBatch gp, gl;  // gl: Lp straight into factor storage (float32 C when f32)
          GemmBatch& glr = f32 ? gl : gp;  // float64 C: one launch for both panels
          std::vector<CopyTask> cps, trs;
          int64_t cu = 0, tu = 0;
          for (auto& e : ep) {
            BoxPlan& bp = plan[e.pi];
            const int m = bp.m, mn = bp.m + bp.nN;
            SolveBox& d = e.fb->dev;
            if (e.nsn > 0) {
              const zd* XsnR = e.Ccol + (int64_t)e.s * mn + e.r;         // X_{(S u N) R}
              const zd* XRsn = e.Crow + e.s + (int64_t)e.r * m;          // X_{R (S u N)}
              e.Up = sg.dev.alloc_n<zd>((size_t)e.r * e.nsn);
              glr.add1(const_cast<void*>(d.Lp), e.nsn, e.nsn, e.r, XsnR, mn, e.Xi64, e.r, e.r, 1.0, 0.0);
              gp.add1(e.Up, e.r, e.r, e.nsn, e.Xi64, e.r, XRsn, m, e.r, 1.0, 0.0);
              trs.push_back(CopyTask{e.Up, const_cast<void*>(d.UpT), e.r, e.nsn, e.r, e.nsn, tu, 1, 0});
              tu += units64(e.r, e.nsn);
            }
            if (e.s > 0) {
              CopyTask c{bp.T, const_cast<void*>(d.T), e.s, e.r, m, e.s, cu};
              cu += units64(e.s, e.r);
              cps.push_back(c);
            }
            if (f32) {
              cps.push_back(CopyTask{e.Xi64, const_cast<void*>(d.Xi), e.r, e.r, e.r, e.r, cu});
              cu += units64(e.r, e.r);
            }
          }
          gp.prepare(sg);
          gl.prepare(sg);
          // the copies and the transposes (of Up, after its product) in one launch
          for (auto& c : trs) {
            c.unit_begin += cu;
            cps.push_back(c);
          }
          CopyTask* dcp = cps.empty() ? nullptr : sg.up(cps);
          ProfScope ps(prof, KC_ELIM);
          gp.launch(sg, 0);
          gl.launch(sg, 0, f32);
          if (dcp) launch_copy(dcp, (int)cps.size(), cu + tu, f32, sg.go());
          for (auto& e : ep) prof.flops[KC_ELIM] += 8.0 * 2.0 * (double)e.nsn * e.r * e.r;
        }
        ht.mark(4);
        // 5. Schur update of near-near tiles: A[SN, SN] -= X_{SN,R} Up. One GEMM task per
        //    destination tile; contributions of several boxes are its segments, in box order.
        {
          // the grouping built while the device computed the IDs, restricted to the boxes that
          // eliminate something (box q = elimination index) and to non-empty contributions
          // (a box without skeleton has none to or from itself); order within tiles is kept
          if (!sg_pre.ok) throw Error(FMMLU_EINVAL, "internal: tile of a pair that is not close");
          std::vector<int> qof(nb, -1);
          for (int q = 0; q < ne; ++q) qof[ep[q].pi] = q;
          bool same = ne == nb;
          for (int q = 0; q < ne && same; ++q) same = ep[q].s > 0;
          std::vector<Contrib> cl_f;
          std::vector<int32_t> first_f;
          if (!same) {
            first_f.push_back(0);
            cl_f.reserve(sg_pre.cl.size());
            for (size_t u = 0; u + 1 < sg_pre.first.size(); ++u) {
              for (int i = sg_pre.first[u]; i < sg_pre.first[u + 1]; ++i) {
                Contrib c = sg_pre.cl[i];
                const int q = qof[c.q];
                if (q < 0 || ((c.a == 0 || c.b == 0) && ep[q].s == 0)) continue;
                c.q = q;
                cl_f.push_back(c);
              }
              if ((int32_t)cl_f.size() > first_f.back()) first_f.push_back((int32_t)cl_f.size());
            }
          }
          std::vector<const std::vector<int>*> grps(ne);
          for (int q = 0; q < ne; ++q) grps[q] = &sg_pre.grps[ep[q].pi];
          const std::vector<Contrib>& cl = same ? sg_pre.cl : cl_f;
          const std::vector<int32_t>& first = same ? sg_pre.first : first_f;
          const int ntk = (int)first.size() - 1;
          // column offsets of the groups in S u N (the box's own skeleton first)
          std::vector<std::vector<int>> goffs(ne);
          for (int q = 0; q < ne; ++q) {
            const std::vector<int>& grp = *grps[q];
            goffs[q].resize(grp.size());
            int off = ep[q].s;
            for (size_t a = 1; a < grp.size(); ++a) {
              goffs[q][a] = off;
              off += (int)own[grp[a]].live.size();
            }
          }
          ht.mark(13);
          // one GEMM task per destination tile with contributions, its segments in box order
          GemmBatch gs;
          gs.tasks.resize(ntk);
          gs.segs.resize(cl.size());
          std::vector<double> tflops(ntk), tbytes(ntk);
          hp.ranges(ntk, 64, [&](int lo, int hi) {
            for (int u = lo; u < hi; ++u) {
              const int i0 = first[u], i1 = first[u + 1];
              double kk = 0;
              for (int i = i0; i < i1; ++i) {
                const Contrib& c = cl[i];
                const ElimPlan& e = ep[c.q];
                const int mn = plan[e.pi].m + plan[e.pi].nN;
                gs.segs[i] = GemmSeg{e.Ccol + (int64_t)e.s * mn + e.r + goffs[c.q][c.a],
                                     e.Up + (int64_t)goffs[c.q][c.b] * e.r, mn, e.r, e.r, 0};
                kk += e.r;
              }
              const Contrib& c0 = cl[i0];
              const ElimPlan& e0 = ep[c0.q];
              const BoxPlan& bp0 = plan[e0.pi];
              const int o1 = (*grps[c0.q])[c0.a], o2 = (*grps[c0.q])[c0.b];
              GemmTask t{};
              t.C = static_cast<char*>(pool) + (size_t)c0.toff * te;
              t.ldc = (int)own[o1].act.size();
              t.M = (c0.a == 0) ? e0.s : (int)own[o1].live.size();
              t.N = (c0.b == 0) ? e0.s : (int)own[o2].live.size();
              t.rmap = (c0.a == 0) ? bp0.perm : own[o1].live_dev;
              t.cmap = (c0.b == 0) ? bp0.perm : own[o2].live_dev;
              t.seg_begin = i0;
              t.nseg = i1 - i0;
              t.alpha_re = -1.0;
              t.alpha_im = 0.0;
              t.beta = 1.0;
              gs.tasks[u] = t;
              tflops[u] = 8.0 * t.M * t.N * kk;
              tbytes[u] = 2.0 * (double)te * t.M * t.N;
            }
          });
          for (int u = 0; u < ntk; ++u) {
            gs.tasks[u].unit_begin = gs.units;
            gs.units += gemm_units(gs.tasks[u].M, gs.tasks[u].N);
            prof.flops[KC_SCHUR] += tflops[u];
            prof.bytes[KC_SCHUR] += tbytes[u];
          }
          for (auto& e : ep) prof.bytes[KC_SCHUR] += 32.0 * (double)e.nsn * e.r;
          ht.mark(14);
          gs.prepare(sg);
          if (!gs.tasks.empty()) {  // a bracket per kernel launch (the launch count is reported)
            ProfScope ps(prof, KC_SCHUR);
            gs.launch(sg, 0, f32);
          }
        }
        // flops of this phase
        for (auto& e : ep) {
          BoxPlan& bp = plan[e.pi];
          info.flops_schur += 8.0 * (double)e.nsn * e.nsn * e.r;
          info.flops_elim += 8.0 * ((double)(bp.m + bp.nN) * e.r * e.s * 2 + 2.0 * e.r * e.r * e.r +
                                   2.0 * e.nsn * e.r * e.r);
        }
      }
      for (auto& bp : plan) {
        const double L = bp.rows, m = bp.m;
        info.flops_id += 8.0 * (2.0 * L * m * std::min(L, m)) + 8.0 * m * m * m;
      }
      // ---- update live lists of eliminated boxes (skeletons in tree order)
      for (int q = 0; q < ne; ++q) {
        ElimPlan& e = ep[q];
        Owner& B = own[plan[e.pi].oi];
        const std::vector<int32_t>& pv = perms[e.pi];
        std::vector<int32_t> nl(pv.begin(), pv.begin() + e.s);
        std::sort(nl.begin(), nl.end());
        B.live = nl;
        live_total -= e.r;
        if (!pos_live.empty())
          for (int j = e.s; j < (int)pv.size(); ++j) pos_live[(size_t)B.act[pv[j]]] = 0;
        info.nboxes_factored++;
      }
      ht.mark(5);
      // build the solve phase record
      if (ne > 0) {
        pending.emplace_back();
        PendingPhase& pp = pending.back();
        SolvePhase& ph = pp.ph;
        ph.box_begin = (int)box_base;
        ph.box_end = (int)boxes.size();
        int64_t yo = 0, po = 0, xpo = 0;
        auto& contrib = pp.contrib;
        auto& db = pp.db;
        auto &txr = pp.txr, &ty = pp.ty, &tbp = pp.tbp, &tbt = pp.tbt, &tbt16 = pp.tbt16;
        auto &txr16 = pp.txr16, &ty16 = pp.ty16, &tbp16 = pp.tbp16, &txs = pp.txs;
        double reread = 0;  // partial entries the blocked 16-row items would read, all items
        for (int b = ph.box_begin; b < ph.box_end; ++b) {
          FactorBox& fb = boxes[b];
          const int lb = b - ph.box_begin;
          SolveBox& d = fb.dev;
          fb.y_off = yo;
          d.y_off = yo;
          d.p_off = po;
          d.xrp_off = xpo;
          d.nks = (fb.s + kSolveK - 1) / kSolveK;
          d.nchunk = (fb.nsn + kSolveK - 1) / kSolveK;
          d.dx_off = dxlen;
          dxlen += fb.r;
          const int ngrp = (fb.r + kSolveOut - 1) / kSolveOut, ngrp16 = (fb.r + 15) / 16;
          for (int c = 0; c < d.nks; ++c) {
            for (int g = 0; g < ngrp; ++g)
              txr.push_back(SweepTask{lb, c * kSolveK, std::min(kSolveK, fb.s - c * kSolveK), c, g, 0});
            for (int g = 0; g < ngrp16; ++g)
              txr16.push_back(SweepTask{lb, c * kSolveK, std::min(kSolveK, fb.s - c * kSolveK), c, g, 0});
          }
          // rows of S u N (forward) and of S (backward), 64 per item; the item of rows 0..63
          // also stores x_R, so a box without such rows still gets one (empty) item
          for (int k0 = 0; k0 < std::max(fb.nsn, 1); k0 += kSolveRows)
            ty.push_back(SweepTask{lb, k0, std::max(0, std::min(kSolveRows, fb.nsn - k0)), 0, 0, 0});
          for (int k0 = 0; k0 < std::max(fb.nsn, 1); k0 += 16)
            ty16.push_back(SweepTask{lb, k0, std::max(0, std::min(16, fb.nsn - k0)), 0, 0, 0});
          for (int c = 0; c < d.nchunk; ++c) {
            for (int g = 0; g < ngrp; ++g)
              tbp.push_back(SweepTask{lb, c * kSolveK, std::min(kSolveK, fb.nsn - c * kSolveK), c, g, 0});
            for (int g = 0; g < ngrp16; ++g)
              tbp16.push_back(SweepTask{lb, c * kSolveK, std::min(kSolveK, fb.nsn - c * kSolveK), c, g, 0});
          }
          for (int l0 = 0; l0 < std::max(fb.s, 1); l0 += kSolveRows)
            tbt.push_back(SweepTask{lb, l0, std::max(0, std::min(kSolveRows, fb.s - l0)), 0, 0, 0});
          for (int l0 = 0; l0 < std::max(fb.s, 1); l0 += 16)
            tbt16.push_back(SweepTask{lb, l0, std::max(0, std::min(16, fb.s - l0)), 0, 0, 0});
          for (int k0 = 0; k0 < fb.r; k0 += kSolveRows)
            txs.push_back(SweepTask{lb, k0, std::min(kSolveRows, fb.r - k0), 0, 0, 0});
          reread += (double)((std::max(fb.s, 1) + 15) / 16) * fb.r * d.nchunk;
          ph.rmax = std::max(ph.rmax, fb.r);
          ph.smax = std::max(ph.smax, fb.s);
          db.push_back(d);
          yo += fb.nsn;
          po += (int64_t)d.nchunk * fb.r;
          xpo += (int64_t)d.nks * fb.r;
        }
        // past 8 MiB of re-read partials (blocks of kSolveBlock complex128), one summing launch
        // is cheaper than the re-reads
        ph.blk_presum = reread * kSolveBlock * sizeof(zd) > 8.0 * (1 << 20);
        // scatter lists: every S u N position of every box of the phase, summed in box order
        for (int q = 0; q < ne; ++q) {
          ElimPlan& e = ep[q];
          BoxPlan& bp = plan[e.pi];
          Owner& B = own[bp.oi];
          const std::vector<int32_t>& pv = perms[e.pi];
          FactorBox& fb = boxes[box_base + q];
          int64_t c = fb.y_off;
          for (int j = 0; j < e.s; ++j) contrib.emplace_back((int32_t)B.act[pv[j]], c++);
          for (int o : bp.nown_)
            for (int32_t l : own[o].live) contrib.emplace_back((int32_t)own[o].act[l], c++);
        }
        if ((size_t)ph.rmax * sizeof(zd) > 65536)
          throw Error(FMMLU_EINVAL, "redundant set of " + std::to_string(ph.rmax) +
                                        " DOFs exceeds the solve kernels' LDS bound (4096)");
        ph.ylen = yo;
        ph.plen = po;
        ph.xrplen = xpo;
        ymax = std::max(ymax, yo);
        pmax = std::max(pmax, po);
        xrpmax = std::max(xrpmax, xpo);
        bgw.post([&pp] { group_scatter(pp); });
      }
      // live lists of eliminated boxes to the device (persistent for the level)
      {
        std::vector<int32_t> live_cat;
        std::vector<int64_t> live_off(ne, -1);
        for (int q = 0; q < ne; ++q) {
          Owner& B = own[plan[ep[q].pi].oi];
          if (B.live.empty()) continue;
          live_off[q] = (int64_t)live_cat.size();
          live_cat.insert(live_cat.end(), B.live.begin(), B.live.end());
        }
        int32_t* live_base = live_cat.empty() ? nullptr : sg.up_to(level_arena, live_cat);
        for (int q = 0; q < ne; ++q) {
          Owner& B = own[plan[ep[q].pi].oi];
          B.live_dev = live_off[q] < 0 ? nullptr : live_base + live_off[q];
        }
      }
      for (auto& bp : plan) info.max_block = std::max(info.max_block, bp.m);
    }
    if (opts.verbose)
      fprintf(stderr, "[fmmlu] level %d: owners %d pairs %zu%s tiles %.1f MB live %lld\n", lev, nown,
              pairs.size(), spec_hit ? " (close lists from the worker)" : "", pool_elems * 16.0 / 1e6,
              (long long)live_total);

    ht.mark(6);
    // ---- next level's owners: merge live DOFs of level-lev owners into parents
    std::vector<Owner> next;
    std::vector<int32_t> next_by_box(tree.nboxes(), -1);  // box -> index in next
    for (int i = 0; i < nown; ++i) {
      Owner& o = own[i];
      if (o.live.empty()) continue;
      int target_box = o.level == lev ? tree.parent[o.box] : o.box;
      int ni = next_by_box[target_box];
      if (ni < 0) {
        ni = (int)next.size();
        next_by_box[target_box] = ni;
        Owner no;
        no.box = target_box;
        no.level = tree.level[target_box];
        no.c[0] = tree.cx[target_box];
        no.c[1] = tree.cy[target_box];
        no.c[2] = tree.cz[target_box];
        no.first_pos = o.act[o.live[0]];
        next.push_back(std::move(no));
      }
      Owner& no = next[ni];
      no.sub.push_back(i);
      for (int32_t l : o.live) no.act.push_back(o.act[l]);
    }
    for (auto& no : next) {
      // sub-owners are visited in tree order, so act is sorted; first_pos = act[0]
      no.first_pos = no.act.front();
    }
    std::sort(next.begin(), next.end(), [](const Owner& a, const Owner& b) { return a.first_pos < b.first_pos; });
    prev_own = std::move(own);
    prev_pidx = std::move(pidx);
    prev_pool = pool;
    own = std::move(next);
    first_level = false;
  }

  ht.mark(7);
  Clock::time_point tt[6];
  tt[0] = Clock::now();
  // ---- top block: all remaining live DOFs (tree order)
  {
    // own holds the owners after the last merge; their act lists are all live.
    std::vector<int32_t> slot, idx;
    std::vector<int64_t> dof;
    std::vector<int32_t> top;
    int nsub = 0;
    if (first_level) {
      // no level was processed (tree with fewer than 3 levels): the top block is A~ itself
      for (auto& o : own) {
        for (int64_t a : o.act) {
          slot.push_back(0);
          idx.push_back(0);
          dof.push_back(a);
        }
      }
      nsub = 1;
    } else {
      nsub = (int)prev_own.size();
      for (size_t q = 0; q < prev_own.size(); ++q) {
        const Owner& so = prev_own[q];
        for (int32_t l : so.live) {
          slot.push_back((int32_t)q);
          idx.push_back(l);
          dof.push_back(so.act[l]);
        }
      }
    }
    n0 = (int)dof.size();
    info.n0 = n0;
    for (int64_t d : dof) top.push_back((int32_t)d);
    if (n0 > 0) {
      std::vector<AsmSrc> table;
      if (first_level) {
        table.push_back(AsmSrc{-1, 0, 0});
      } else {
        const int64_t np = (int64_t)prev_own.size();
        table.resize((size_t)np * np, AsmSrc{-1, 0, 0});
        for (int64_t a = 0; a < np; ++a)
          for (int64_t k = prev_pidx.beg[a]; k < prev_pidx.beg[a + 1]; ++k)
            table[a * np + prev_pidx.ids[k]] = AsmSrc{prev_pidx.off[k], (int32_t)prev_own[a].act.size(), 0};
      }
      zd* Att = sg.dev.alloc_n<zd>((size_t)n0 * n0);
      AsmTask t{};
      t.out_off = 0;
      t.nr = n0;
      t.nc = n0;
      t.ld = n0;
      t.nsc = first_level ? 1 : nsub;
      t.rmap_off = 0;
      t.cmap_off = 0;
      t.rdof_off = 0;
      t.cdof_off = 0;
      t.tab_off = 0;
      t.unit_begin = 0;
      std::vector<AsmTask> tv{t};
      {
        AsmTask* dt = sg.up(tv);
        int32_t* dslot = sg.up(slot);
        int32_t* didx = sg.up(idx);
        int64_t* ddof = sg.up(dof);
        AsmSrc* dtab = sg.up(table);
        ProfScope ps(prof, KC_TOP);
        launch_assemble(g, dt, 1, units64(n0, n0), dslot, didx, ddof, dtab, prev_pool, f32, Att, false, sg.go());
      }
      Ainv = arena.alloc_n<zd>((size_t)n0 * n0);
      std::vector<GjTask> gt(1);
      gt[0].A = Att;
      gt[0].n = n0;
      gt[0].lda = n0;
      std::vector<zd*> outs{Ainv};
      batched_inverse(sg, gt, outs, info_dev, KC_TOP);
      top_dev = sg.up_to(arena, top);
      tt[1] = Clock::now();
      info.flops_top = 8.0 * (double)n0 * n0 * n0;
      info.factor_bytes += 16 * (int64_t)n0 * n0;
    }
    // solve records: the scatter lists were grouped on the background worker while the
    // planning thread waited on the device; all arrays of all phases leave in one copy
    if (n0 <= 0) tt[1] = Clock::now();
    bgw.drain();
    tt[2] = Clock::now();
    {
      std::vector<SolvePhase> newph(pending.size());
      Stage::Packed pk;
      size_t i = 0;
      for (PendingPhase& pp : pending) {
        SolvePhase& ph = newph[i++];
        ph = pp.ph;
        ph.nd = (int64_t)pp.dst.size();
        ph.direct = pp.src.size() == pp.dst.size();
        pk.add(&ph.dboxes, pp.db);
        pk.add(&ph.sc_dst, pp.dst);
        pk.add(&ph.sc_ptr, pp.ptr);
        pk.add(&ph.sc_src, pp.src);
        pk.add(&ph.dbt16, pp.tbt16);
        pk.add(&ph.dxs, pp.txs);
        ph.nxs = (int)pp.txs.size();
        ph.nxr = (int)pp.txr.size();
        ph.ny = (int)pp.ty.size();
        ph.nbp = (int)pp.tbp.size();
        ph.nbt = (int)pp.tbt.size();
        ph.nbt16 = (int)pp.tbt16.size();
        // items of 16 outputs or rows where the items of 64 would leave most compute units idle
        auto pick = [&](SweepTask** dst, int* cnt, int* gran, const std::vector<SweepTask>& coarse,
                        const std::vector<SweepTask>& fine16, int coarse_gran) {
          const bool f = (int)coarse.size() < kSolveFineBelow;
          pk.add(dst, f ? fine16 : coarse);
          *cnt = (int)(f ? fine16 : coarse).size();
          *gran = f ? 16 : coarse_gran;
        };
        pick(&ph.s1xr, &ph.n1xr, &ph.g1xr, pp.txr, pp.txr16, kSolveOut);
        pick(&ph.s1y, &ph.n1y, &ph.g1y, pp.ty, pp.ty16, kSolveRows);
        pick(&ph.s1bp, &ph.n1bp, &ph.g1bp, pp.tbp, pp.tbp16, kSolveOut);
        pick(&ph.s1bt, &ph.n1bt, &ph.g1bt, pp.tbt, pp.tbt16, kSolveRows);
      }
      sg.commit(arena, pk);
      if (opts.verbose) {
        int nf[4] = {0, 0, 0, 0}, maxc[4] = {0, 0, 0, 0}, npre = 0;
        int ndirect = 0;
        for (auto& ph : newph) {
          npre += ph.blk_presum;
          ndirect += ph.direct;
          nf[0] += ph.g1xr == 16; nf[1] += ph.g1y == 16; nf[2] += ph.g1bp == 16; nf[3] += ph.g1bt == 16;
          maxc[0] = std::max(maxc[0], ph.nxr); maxc[1] = std::max(maxc[1], ph.ny);
          maxc[2] = std::max(maxc[2], ph.nbp); maxc[3] = std::max(maxc[3], ph.nbt);
        }
        fprintf(stderr, "[fmmlu] sweeps: phases with 16-wide items (of %zu) xr %d y %d bpart %d bt %d; "
                "most 64-wide items in a phase %d %d %d %d; blocked sweeps summing x_R per phase: %d\n", newph.size(),
                nf[0], nf[1], nf[2], nf[3], maxc[0], maxc[1], maxc[2], maxc[3], npre);
        fprintf(stderr, "[fmmlu] sweeps: phases without a shared row of S u N (no scatter launch): %d\n", ndirect);
      }
      for (auto& ph : newph) phases.push_back(ph);
    }
    pending.clear();
    // the table of all boxes, then the forward and adjoint solve graphs, captured while the
    // top block is still running (a capture only records launches)
    {
      std::vector<SolveBox> all;
      std::vector<SweepTask> dg;
      for (auto& fb : boxes) {
        for (int i0 = 0; i0 < fb.r; i0 += kSolveOut)
          dg.push_back(SweepTask{(int32_t)all.size(), i0, std::min(kSolveOut, fb.r - i0), 0, 0, 0});
        all.push_back(fb.dev);
        rmax_all = std::max(rmax_all, fb.r);
      }
      nall = (int)all.size();
      all_boxes = sg.up_to(arena, all);
      ndg = (int)dg.size();
      dg_tasks = sg.up_to(arena, dg);
    }
    tt[3] = Clock::now();
    if (use_graph && precapture && ActiveFactorization::count() == 1) {
      ensure_workspace();
      if (!capture(0) || !capture(1)) use_graph = false;
    }
    tt[4] = Clock::now();
    sg.sync_reset();
    tt[5] = Clock::now();
    prev_pool = nullptr;
    // the first zero pivot of any pivot block or of the top block (column + 1), or -1 if a
    // cooperative barrier timed out
    int32_t hinfo = 0;
    FMMLU_HIP(hipMemcpyAsync(&hinfo, info_dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMMLU_HIP(hipStreamSynchronize(st));
    if (hinfo < 0) throw Error(FMMLU_EHIP, "Gauss-Jordan panel barrier timed out");
    if (hinfo != 0) throw Error(FMMLU_ESINGULAR, "singular pivot block (X_RR or the top block)");
  }
  info.peak_bytes = (int64_t)mem.peak();
  info.t_factor = std::chrono::duration<double>(Clock::now() - t0).count();
  if (opts.verbose) {
    fprintf(stderr, "[fmmlu] factor %.3f s, of which waiting on the GPU %.3f s\n", info.t_factor, sg.t_wait);
    fprintf(stderr,
            "[fmmlu] host sections: pairs %.3f pool %.3f assemble %.3f plan %.3f id+readback %.3f elim %.3f "
            "schur %.3f phase-end %.3f merge %.3f\n",
            ht.t[0], ht.t[8], ht.t[1], ht.t[2], ht.t[3], ht.t[4], ht.t[5], ht.t[6], ht.t[7]);
    fprintf(stderr, "[fmmlu] elimination planning: boxes %.3f cross %.3f E/F %.3f inverse %.3f panels %.3f\n",
            ht.t[9], ht.t[10], ht.t[11], ht.t[12], ht.t[4]);
    auto ms = [&](int a, int b) { return std::chrono::duration<double, std::milli>(tt[b] - tt[a]).count(); };
    fprintf(stderr, "[fmmlu] tail (ms): top block planning+launch %.2f, record grouping wait %.2f, records upload %.2f, "
            "graph capture %.2f, final wait %.2f\n", ms(0, 1), ms(1, 2), ms(2, 3), ms(3, 4), ms(4, 5));
    fprintf(stderr, "[fmmlu] schur planning: contributions %.3f tasks %.3f launch+rest %.3f\n", ht.t[13], ht.t[14],
            ht.t[5]);
    fprintf(stderr, "[fmmlu] blocked pivoting continued past the rank bound in %d phases\n", pchol_continued);
  }
}

// ------------------------------------------------------------------------------------------
void FactorImpl::alloc_ws(SolveWs& w, int nr) {
  auto al = [&](int64_t len) { return arena.alloc_n<zd>((size_t)std::max<int64_t>(len, 1) * (size_t)nr); };
  const int64_t nblk = (n0 + 255) / 256;
  w.x = al(n);
  w.y = al(ymax);
  w.p = al(pmax);
  w.xrp = al(xrpmax);
  w.xrg = al(dxlen);
  w.xrd = al(dxlen);
  w.top = al((int64_t)n0 * (1 + nblk));
}

void FactorImpl::ensure_workspace() {
  if (ws1.x) return;
  alloc_ws(ws1, 1);
  wmv = arena.alloc_n<zd>((size_t)n);
  wpart_entries = (int64_t)matvec_slices(n) * n;
  wpart = arena.alloc_n<zd>((size_t)wpart_entries);
}

void FactorImpl::solve_core(const zd* bc, zd* xc, bool adjoint, hipStream_t st) {
  sweep(ws1, 1, bc, n, xc, n, 1, adjoint, st);
}

void FactorImpl::sweep(const SolveWs& w, int nr, const zd* bc, int64_t ldb, zd* xc, int64_t ldx, int m,
                       bool adjoint, hipStream_t st) {
  const int adj = adjoint ? 1 : 0;
  const bool blk = nr == kSolveBlock;
  if (!blk && nr != 1) throw Error(FMMLU_EINVAL, "sweep of " + std::to_string(nr) + " columns");
  launch_permute(bc, w.x, order_dev, n, 1, st, nr, ldb, m);
  // V_1^{-1} ... V_M^{-1} (adjoint: W_1^{-H} ... W_M^{-H}), phase by phase: x_R partials, then
  // x_R and the updates y of S u N, then their deterministic sum into x
  for (auto& ph : phases) {
    if (blk) {
      launch_blk_xr_part(ph.dboxes, ph.s1xr, ph.n1xr, ph.g1xr, w.x, w.xrp, adj, f32, st);
      launch_blk_y(ph.dboxes, ph.s1y, ph.n1y, ph.g1y, w.x, w.xrp, w.xrg, w.y, adj, ph.direct, f32, st);
    } else {
      launch_solve_xr_part(ph.dboxes, ph.s1xr, ph.n1xr, ph.g1xr, w.x, w.xrp, adj, f32, st, nr);
      launch_solve_y(ph.dboxes, ph.s1y, ph.n1y, ph.g1y, w.x, w.xrp, w.xrg, w.y, adj, ph.direct, f32, st, nr);
    }
    if (!ph.direct) launch_scatter_sub(ph.sc_dst, ph.sc_ptr, ph.sc_src, ph.nd, w.y, w.x, st, nr);
  }
  // D^{-1} (adjoint D^{-H}): all pivot blocks (x_R buffer to x_R buffer), then the top block
  if (blk) {
    launch_blk_diag(all_boxes, dg_tasks, ndg, w.xrg, w.xrd, adj, f32, st);
    launch_solve_top_gather(n0, top_dev, w.x, w.top, st, nr);
    launch_blk_top_part(Ainv, n0, w.top, w.top + (int64_t)n0 * nr, adj, st);
    launch_solve_top_fin(n0, top_dev, w.top + (int64_t)n0 * nr, w.x, st, nr);
  } else {
    launch_solve_diag(all_boxes, dg_tasks, ndg, rmax_all, w.xrg, w.xrd, adj, f32, st, nr);
    launch_solve_top(Ainv, n0, top_dev, w.x, w.top, adj, st, nr);
  }
  // W_M^{-1} ... W_1^{-1} (adjoint: V_M^{-H} ... V_1^{-H}), phases in reverse: x_R partials,
  // then x_R into x and the updates of x_S
  for (auto it = phases.rbegin(); it != phases.rend(); ++it) {
    if (blk) {
      launch_blk_bpart(it->dboxes, it->s1bp, it->n1bp, it->g1bp, w.x, w.p, adj, f32, st);
      if (it->blk_presum) launch_blk_xr_sub(it->dboxes, it->dxs, it->nxs, w.xrd, w.p, w.x, st);
      launch_blk_bt(it->dboxes, it->dbt16, it->nbt16, w.xrd, w.p, w.x, adj, it->blk_presum, f32, st);
    } else {
      launch_solve_bpart(it->dboxes, it->s1bp, it->n1bp, it->g1bp, w.x, w.p, adj, f32, st, nr);
      launch_solve_bt(it->dboxes, it->s1bt, it->n1bt, it->g1bt, w.xrd, w.p, w.x, adj, f32, st, nr);
    }
  }
  launch_permute(w.x, xc, order_dev, n, 0, st, nr, ldx, m);
}

// the blocked sweeps stage x_R in chunks: no bound on the redundant sets
bool FactorImpl::blocked_ok() const { return true; }

void FactorImpl::ensure_block_workspace() {
  if (wsb.x) return;
  alloc_ws(wsb, kSolveBlock);
  ginb = arena.alloc_n<zd>((size_t)n * kSolveBlock);
  goutb = arena.alloc_n<zd>((size_t)n * kSolveBlock);
}

// the blocked sweeps of one direction in a graph on the private stream (ginb -> goutb)
bool FactorImpl::capture_block(int adj) {
  if (gexecb[adj]) return true;
  if (!gstream) FMMLU_HIP(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking));
  if (hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = true;
  try {
    sweep(wsb, kSolveBlock, ginb, n, goutb, n, kSolveBlock, adj != 0, gstream);
  } catch (const Error&) {
    ok = false;
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(gstream, &g) != hipSuccess || !ok || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return false;
  }
  graphb[adj] = g;
  gexecb[adj] = e;
  return true;
}

// Capture the sweeps of one direction into a graph on a private stream (reading gin,
// writing gout). The sweeps contain kernels only: no copies, fills or allocations.
bool FactorImpl::capture(int adj) {
  if (gexec[adj]) return true;
  if (!gstream) FMMLU_HIP(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking));
  if (!gin) {
    gin = arena.alloc_n<zd>((size_t)n);
    gout = arena.alloc_n<zd>((size_t)n);
  }
  if (hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = true;
  try {
    solve_core(gin, gout, adj != 0, gstream);
  } catch (const Error&) {
    ok = false;
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(gstream, &g) != hipSuccess || !ok || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return false;
  }
  graph[adj] = g;
  gexec[adj] = e;
  return true;
}

void FactorImpl::solve(const zd* b, zd* x, int64_t nrhs, bool adjoint, hipStream_t st) {
  ensure_workspace();
  const int adj = adjoint ? 1 : 0;
  if (nrhs > 1 && blocked_ok()) {
    // blocks of kSolveBlock columns: every factor entry is read once per block
    ensure_block_workspace();
    const bool g = use_graph && capture_block(adj);
    for (int64_t c0 = 0; c0 < nrhs; c0 += kSolveBlock) {
      const int m = (int)std::min<int64_t>(kSolveBlock, nrhs - c0);
      const zd* bc = b + c0 * n;
      zd* xc = x + c0 * n;
      if (g) {
        FMMLU_HIP(hipMemcpyAsync(ginb, bc, sizeof(zd) * (size_t)(n * m), hipMemcpyDeviceToDevice, st));
        if (m < kSolveBlock)
          FMMLU_HIP(hipMemsetAsync(ginb + n * m, 0, sizeof(zd) * (size_t)(n * (kSolveBlock - m)), st));
        FMMLU_HIP(hipGraphLaunch(gexecb[adj], st));
        FMMLU_HIP(hipMemcpyAsync(xc, goutb, sizeof(zd) * (size_t)(n * m), hipMemcpyDeviceToDevice, st));
      } else {
        sweep(wsb, kSolveBlock, bc, n, xc, n, m, adjoint, st);
      }
    }
    return;
  }
  const bool g = use_graph && capture(adj);
  if (!g) use_graph = false;
  for (int64_t c = 0; c < nrhs; ++c) {
    const zd* bc = b + c * n;
    zd* xc = x + c * n;
    if (g) {
      FMMLU_HIP(hipMemcpyAsync(gin, bc, sizeof(zd) * (size_t)n, hipMemcpyDeviceToDevice, st));
      FMMLU_HIP(hipGraphLaunch(gexec[adj], st));
      FMMLU_HIP(hipMemcpyAsync(xc, gout, sizeof(zd) * (size_t)n, hipMemcpyDeviceToDevice, st));
    } else {
      solve_core(bc, xc, adjoint, st);
    }
  }
}

FactorImpl::~FactorImpl() {
  // solves may still be running on any stream; the arenas are freed after the device drains
  (void)hipDeviceSynchronize();
  for (int a = 0; a < 2; ++a) {
    if (gexecb[a]) (void)hipGraphExecDestroy(gexecb[a]);
    if (graphb[a]) (void)hipGraphDestroy(graphb[a]);
    if (gexec[a]) (void)hipGraphExecDestroy(gexec[a]);
    if (graph[a]) (void)hipGraphDestroy(graph[a]);
  }
  if (gstream) (void)hipStreamDestroy(gstream);
}

}  // namespace fmmlu
