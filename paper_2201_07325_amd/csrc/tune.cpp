// GEMM autotuning: for every use of the batched GEMM (precision, mapped output, op(A)) and
// every K bucket, each kernel that implements it is timed once per device and process on a
// synthetic batch of that bucket's shape, and later launches in the bucket use the fastest.
// A candidate replaces the default kernel only when it is more than kMargin faster (best of
// five launches each), so that timing noise rarely flips the choice (and with it the
// rounding) between processes; within a process the choice is fixed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tune.hpp"

namespace fmmlu {

namespace {

constexpr int kBuckets = 3;                       // K <= 32, K <= 512, larger
constexpr int kBucketK[kBuckets] = {16, 256, 2048};  // K of each bucket's timing batch
constexpr int kTuneTasks = 32, kTuneM = 192;       // batch: 32 products with 192 x 192 outputs
constexpr double kMargin = 0.10;

struct Use {
  bool c32, mapped;
  int opA;
};
// the uses the library launches, and the kernels that implement each
const Use kUses[] = {{false, true, 0}, {false, false, 0}, {false, false, 1}, {false, false, 2},
                     {true, true, 0},  {true, false, 0}};
constexpr int kNumUses = sizeof(kUses) / sizeof(kUses[0]);

std::vector<int> candidates(const Use&) { return {GK_LDS, GK_REG8, GK_REG4}; }

struct Table {
  bool done = false;
  int choice[kNumUses][kBuckets];
  float ms[kNumUses][kBuckets][3];  // per kernel id (GK_LDS, GK_REG8, GK_REG4); < 0: not a candidate
};

std::mutex g_mu;
std::vector<Table> g_tables;  // per device

int use_index(bool c32, bool mapped, int opA) {
  for (int i = 0; i < kNumUses; ++i)
    if (kUses[i].c32 == c32 && kUses[i].mapped == mapped && kUses[i].opA == opA) return i;
  return -1;
}

const char* kname(int k) { return k == GK_LDS ? "lds64x8" : k == GK_REG8 ? "reg64x8" : "reg64x4"; }

}  // namespace

thread_local int t_force = GK_AUTO;

int gemm_bucket(int64_t k) { return k <= 32 ? 0 : k <= 512 ? 1 : 2; }

void gemm_force_kernel(int kernel) { t_force = kernel; }

int gemm_tuned_kernel(bool c32, bool mapped, int opA, int64_t kmax) {
  if (t_force != GK_AUTO) return t_force;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GK_AUTO;
  std::lock_guard<std::mutex> l(g_mu);
  if (dev >= (int)g_tables.size() || !g_tables[dev].done) return GK_AUTO;
  const int u = use_index(c32, mapped, opA);
  return u < 0 ? GK_AUTO : g_tables[dev].choice[u][gemm_bucket(kmax)];
}

void gemm_autotune(DeviceMemory& mem, hipStream_t st) {
  int dev = 0;
  FMMLU_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> l(g_mu);
  if (dev >= (int)g_tables.size()) g_tables.resize(dev + 1);
  Table& tb = g_tables[dev];
  if (tb.done) return;
  const int M = kTuneM, T = kTuneTasks, Kmax = kBucketK[kBuckets - 1];
  // operands shared by the batch (finite values), one output block per product
  const size_t ab = sizeof(zd) * (size_t)M * Kmax, cb = sizeof(zd) * (size_t)M * M * T;
  size_t ga = 0, gb = 0, gc = 0, gm = 0, gt = 0;
  void* A = mem.get(ab, ga);
  void* B = mem.get(ab, gb);
  void* Cm = mem.get(cb, gc);
  void* maps = mem.get(sizeof(int32_t) * M, gm);
  const size_t desc = sizeof(GemmTask) * T + sizeof(GemmSeg) * T;
  void* dd = mem.get(desc, gt);
  struct Release {
    DeviceMemory& m;
    std::vector<std::pair<void*, size_t>> b;
    ~Release() {
      for (auto& x : b) m.put(x.first, x.second);
    }
  } rel{mem, {{A, ga}, {B, gb}, {Cm, gc}, {maps, gm}, {dd, gt}}};
  {
    std::vector<zd> h((size_t)M * Kmax);
    for (size_t i = 0; i < h.size(); ++i) h[i] = zd{1.0 / (1.0 + (double)(i % 97)), 0.5 / (1.0 + (double)(i % 89))};
    FMMLU_HIP(hipMemcpyAsync(A, h.data(), ab, hipMemcpyHostToDevice, st));
    FMMLU_HIP(hipMemcpyAsync(B, h.data(), ab, hipMemcpyHostToDevice, st));
    FMMLU_HIP(hipMemsetAsync(Cm, 0, cb, st));
    std::vector<int32_t> id(M);
    for (int i = 0; i < M; ++i) id[i] = i;
    FMMLU_HIP(hipMemcpyAsync(maps, id.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, st));
    FMMLU_HIP(hipStreamSynchronize(st));
  }
  hipEvent_t e0, e1;
  FMMLU_HIP(hipEventCreate(&e0));
  FMMLU_HIP(hipEventCreate(&e1));
  const int64_t tiles = gemm_task_tiles(M, M, false);
  for (int ui = 0; ui < kNumUses; ++ui) {
    const Use& u = kUses[ui];
    const int def = gemm_default_kernel(u.c32, u.mapped, u.opA);
    for (int bk = 0; bk < kBuckets; ++bk) {
      const int K = kBucketK[bk];
      std::vector<GemmTask> tasks(T);
      std::vector<GemmSeg> segs(T);
      const size_t csz = u.c32 ? sizeof(zf) : sizeof(zd);
      for (int i = 0; i < T; ++i) {
        GemmTask t{};
        t.C = static_cast<char*>(Cm) + csz * (size_t)M * M * i;
        t.rmap = u.mapped ? static_cast<const int32_t*>(maps) : nullptr;
        t.cmap = u.mapped ? static_cast<const int32_t*>(maps) : nullptr;
        t.M = M;
        t.N = M;
        t.ldc = M;
        t.seg_begin = i;
        t.nseg = 1;
        t.alpha_re = 1.0;
        t.beta = 1.0;
        t.unit_begin = tiles * i;
        tasks[i] = t;
        // op(A) is M x K: stored M x K (opA = 0) or K x M (transposed)
        segs[i] = GemmSeg{static_cast<const zd*>(A), static_cast<const zd*>(B), u.opA == 0 ? M : K, K, K, 0};
      }
      GemmTask* dtk = static_cast<GemmTask*>(dd);
      GemmSeg* dsg = reinterpret_cast<GemmSeg*>(static_cast<char*>(dd) + sizeof(GemmTask) * T);
      FMMLU_HIP(hipMemcpyAsync(dtk, tasks.data(), sizeof(GemmTask) * T, hipMemcpyHostToDevice, st));
      FMMLU_HIP(hipMemcpyAsync(dsg, segs.data(), sizeof(GemmSeg) * T, hipMemcpyHostToDevice, st));
      float best = 1e30f, tdef = -1.0f;
      int bestk = def;
      for (int k = 0; k < 3; ++k) tb.ms[ui][bk][k] = -1.0f;
      for (int k : candidates(u)) {
        launch_gemm(u.opA, dtk, T, tiles * T, dsg, u.c32, st, u.mapped, nullptr, k);  // warm-up
        float tmin = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
          FMMLU_HIP(hipEventRecord(e0, st));
          launch_gemm(u.opA, dtk, T, tiles * T, dsg, u.c32, st, u.mapped, nullptr, k);
          FMMLU_HIP(hipEventRecord(e1, st));
          FMMLU_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          FMMLU_HIP(hipEventElapsedTime(&ms, e0, e1));
          tmin = std::min(tmin, ms);
        }
        tb.ms[ui][bk][k] = tmin;
        if (k == def) tdef = tmin;
        if (tmin < best) {
          best = tmin;
          bestk = k;
        }
      }
      // keep the default unless another kernel is clearly faster
      tb.choice[ui][bk] = (tdef > 0.0f && best > (1.0f - (float)kMargin) * tdef) ? def : bestk;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tb.done = true;
}

std::string gemm_tune_report() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "";
  std::lock_guard<std::mutex> l(g_mu);
  if (dev >= (int)g_tables.size() || !g_tables[dev].done) return "";
  const Table& tb = g_tables[dev];
  std::string s = "{\"batch\": \"32 products, 192 x 192 outputs, K 16 / 256 / 2048\", \"choices\": [";
  char buf[512];
  for (int ui = 0; ui < kNumUses; ++ui)
    for (int bk = 0; bk < kBuckets; ++bk) {
      const Use& u = kUses[ui];
      std::snprintf(buf, sizeof buf,
                    "%s{\"precision\": \"%s\", \"mapped\": %d, \"opA\": %d, \"k_bucket\": \"%s\", \"kernel\": \"%s\", "
                    "\"ms\": {",
                    (ui || bk) ? ", " : "", u.c32 ? "c64" : "c128", u.mapped ? 1 : 0, u.opA,
                    bk == 0 ? "<=32" : bk == 1 ? "<=512" : ">512", kname(tb.choice[ui][bk]));
      s += buf;
      bool first = true;
      for (int k = 0; k < 3; ++k) {
        if (tb.ms[ui][bk][k] < 0.0f) continue;
        std::snprintf(buf, sizeof buf, "%s\"%s\": %.4f", first ? "" : ", ", kname(k), tb.ms[ui][bk][k]);
        s += buf;
        first = false;
      }
      s += "}}";
    }
  s += "]}";
  return s;
}

}  // namespace fmmlu
