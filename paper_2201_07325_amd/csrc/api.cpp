// C ABI of the library: argument validation, handle management, error translation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fmmlu.h"
#include "common.hpp"
#include "batch.hpp"
#include "factor.hpp"
#include "tune.hpp"
#include "kernels.hpp"
#include "tree.hpp"

using namespace fmmlu;

struct fmmlu_tree_s {
  Octree t;
  std::vector<double> xyz;  // copy of the points (for consistency checks in factor)
  double t_build = 0;
};

struct fmmlu_factor_s {
  FactorImpl f;
};

namespace {

thread_local std::string g_last_error;

fmmlu_status fail(fmmlu_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

template <class F>
fmmlu_status guarded(F&& fn) {
  try {
    g_last_error.clear();
    fn();
    return FMMLU_OK;
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(FMMLU_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FMMLU_EINVAL, e.what());
  } catch (...) {
    return fail(FMMLU_EINVAL, "unknown error");
  }
}

void check_finite(const double* v, int64_t cnt, const char* what) {
  for (int64_t i = 0; i < cnt; ++i)
    if (!std::isfinite(v[i])) throw Error(FMMLU_EINVAL, std::string(what) + " contains NaN or Inf");
}

// Checks of fmmlu_factor's arguments that need no GPU; returns the options to use.
fmmlu_opts checked_opts(fmmlu_tree_h t, const double* xyz, const double* normals, const double* weights, double k,
                        double eta, const fmmlu_opts* opts) {
  if (!t) throw Error(FMMLU_ESTATE, "tree is NULL");
  if (!xyz || !normals || !weights) throw Error(FMMLU_EINVAL, "geometry pointer is NULL");
  fmmlu_opts o;
  if (opts)
    o = *opts;
  else
    fmmlu_default_opts(&o);
  if (!(o.eps > 0.0 && o.eps <= 0.1)) throw Error(FMMLU_EINVAL, "eps must be in (0, 0.1]");
  if (!(k >= 0.0) || !std::isfinite(k)) throw Error(FMMLU_EINVAL, "k must be finite and >= 0");
  if (!std::isfinite(eta)) throw Error(FMMLU_EINVAL, "eta must be finite");
  if (!(o.proxy_radius >= 1.5 && o.proxy_radius <= 10.0)) throw Error(FMMLU_EINVAL, "proxy_radius must be in [1.5, 10]");
  if (o.proxy_min_points < 1) throw Error(FMMLU_EINVAL, "proxy_min_points must be >= 1");
  if (o.id_route < 0 || o.id_route > 2) throw Error(FMMLU_EINVAL, "id_route must be 0, 1 or 2");
  if (o.gemm_autotune < 0 || o.gemm_autotune > 4) throw Error(FMMLU_EINVAL, "gemm_autotune must be in 0..4");
  if (o.pchol_blocks < 0) throw Error(FMMLU_EINVAL, "pchol_blocks must be >= 0");
  if ((o.alloc == nullptr) != (o.free == nullptr))
    throw Error(FMMLU_EINVAL, "alloc and free must be given together");
  if ((o.corr_row_ptr == nullptr) != (o.corr_col == nullptr) || (o.corr_row_ptr == nullptr) != (o.corr_a == nullptr))
    throw Error(FMMLU_EINVAL, "corr_row_ptr, corr_col and corr_a must be given together");
  if (o.corr_row_ptr) {
    const int64_t nn = t->t.n;
    if (o.corr_row_ptr[0] != 0) throw Error(FMMLU_EINVAL, "corr_row_ptr[0] must be 0");
    for (int64_t i = 0; i < nn; ++i)
      if (o.corr_row_ptr[i + 1] < o.corr_row_ptr[i]) throw Error(FMMLU_EINVAL, "corr_row_ptr must not decrease");
    for (int64_t e = 0; e < o.corr_row_ptr[nn]; ++e) {
      if (o.corr_col[e] < 0 || o.corr_col[e] >= nn) throw Error(FMMLU_EINVAL, "corr_col entry out of range");
      if (!std::isfinite(o.corr_a[e])) throw Error(FMMLU_EINVAL, "corr_a contains NaN or Inf");
    }
  }
  if (o.precision != FMMLU_FP64 && o.precision != FMMLU_FP32)
    throw Error(FMMLU_EINVAL, "precision must be FMMLU_FP64 or FMMLU_FP32");
  const int64_t n = t->t.n;
  check_finite(xyz, 3 * n, "points");
  check_finite(normals, 3 * n, "normals");
  check_finite(weights, n, "weights");
  if (std::memcmp(xyz, t->xyz.data(), sizeof(double) * 3 * n) != 0)
    throw Error(FMMLU_EINVAL, "points differ from those the tree was built from");
  for (int64_t i = 0; i < n; ++i) {
    if (!(weights[i] > 0.0)) throw Error(FMMLU_EINVAL, "weights must be positive");
    const double nn =
        normals[i] * normals[i] + normals[n + i] * normals[n + i] + normals[2 * n + i] * normals[2 * n + i];
    if (std::fabs(nn - 1.0) > 1e-6) throw Error(FMMLU_EINVAL, "normals must be unit vectors");
  }
  return o;
}

// Factor on the calling thread's current device; the handle owns the result.
// precapture: record the solve graphs at the end of the factorization (not while other
// threads factor: their legacy-stream work may not overlap a capture)
fmmlu_factor_s* make_factor(fmmlu_tree_h t, const double* xyz, const double* normals, const double* weights, double k,
                            double eta, const fmmlu_opts& o, hipStream_t st, bool precapture = true) {
  auto* h = new fmmlu_factor_s;
  try {
    FMMLU_HIP(hipGetDevice(&h->f.device));
    h->f.k = k;
    h->f.eta = eta;
    h->f.opts = o;
    h->f.precapture = precapture;
    h->f.factor(t->t, xyz, normals, weights, st);
    h->f.info.t_tree = t->t_build;
  } catch (...) {
    delete h;
    throw;
  }
  return h;
}

}  // namespace

// ---- batches of independent problems ----
struct fmmlu_batch_s {
  std::vector<fmmlu_factor_s*> factors;  // owned
  std::vector<int64_t> offsets;          // count + 1
  BatchSolver solver;
  ~fmmlu_batch_s() {
    for (auto* f : factors) delete f;
  }
};

extern "C" {

fmmlu_status fmmlu_default_opts(fmmlu_opts* opts) {
  if (!opts) return fail(FMMLU_EINVAL, "opts is NULL");
  std::memset(opts, 0, sizeof(*opts));
  opts->eps = 1e-6;
  opts->proxy_radius = 2.5;
  opts->proxy_min_points = 64;
  opts->precision = FMMLU_FP64;
  opts->device_mem_cap = 0;
  opts->verbose = 0;
  opts->profile = 0;
  opts->id_route = 0;
  opts->test_zero_pivot_block = -1;
  opts->gemm_autotune = 1;
  return FMMLU_OK;
}

fmmlu_status fmmlu_build_tree(const double* xyz, int64_t n, int32_t leaf_size, fmmlu_tree_h* out) {
  if (!out) return fail(FMMLU_EINVAL, "out is NULL");
  *out = nullptr;
  if (!xyz) return fail(FMMLU_EINVAL, "xyz is NULL");
  if (n < 1) return fail(FMMLU_EINVAL, "n must be >= 1");
  if (n > INT32_MAX) return fail(FMMLU_EINVAL, "n must fit in int32");
  if (leaf_size < 1) return fail(FMMLU_EINVAL, "leaf_size must be >= 1");
  return guarded([&] {
    check_finite(xyz, 3 * n, "points");
    auto t0 = std::chrono::steady_clock::now();
    auto* h = new fmmlu_tree_s;
    try {
      h->t.build(xyz, n, leaf_size);
      // duplicate points share a full-depth key; compare coordinates within equal keys
      const auto& ms = h->t.msort;
      for (int64_t i = 1; i < n; ++i) {
        if (h->t.key[ms[i]] != h->t.key[ms[i - 1]]) continue;
        for (int64_t j = i - 1; j >= 0 && h->t.key[ms[j]] == h->t.key[ms[i]]; --j) {
          const int64_t a = ms[i], b = ms[j];
          if (xyz[a] == xyz[b] && xyz[n + a] == xyz[n + b] && xyz[2 * n + a] == xyz[2 * n + b])
            throw Error(FMMLU_EINVAL, "duplicate points " + std::to_string(b) + " and " + std::to_string(a));
        }
      }
      h->xyz.assign(xyz, xyz + 3 * n);
      h->t_build = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

fmmlu_status fmmlu_tree_info(fmmlu_tree_h t, int64_t* nboxes, int32_t* nlevels, int64_t* nleaves) {
  if (!t) return fail(FMMLU_ESTATE, "tree is NULL");
  if (nboxes) *nboxes = t->t.nboxes();
  if (nlevels) *nlevels = t->t.nlevels;
  if (nleaves) {
    int64_t c = 0;
    for (int64_t b = 0; b < t->t.nboxes(); ++b) c += t->t.is_leaf((int)b);
    *nleaves = c;
  }
  return FMMLU_OK;
}

fmmlu_status fmmlu_tree_export(fmmlu_tree_h t, int32_t* level, int32_t* coord, int32_t* npts,
                               int8_t* is_leaf, int64_t* order) {
  if (!t) return fail(FMMLU_ESTATE, "tree is NULL");
  const Octree& o = t->t;
  for (int64_t b = 0; b < o.nboxes(); ++b) {
    if (level) level[b] = o.level[b];
    if (coord) {
      coord[3 * b] = o.cx[b];
      coord[3 * b + 1] = o.cy[b];
      coord[3 * b + 2] = o.cz[b];
    }
    if (npts) npts[b] = (int32_t)o.npts((int)b);
    if (is_leaf) is_leaf[b] = o.is_leaf((int)b) ? 1 : 0;
  }
  if (order)
    for (int64_t i = 0; i < o.n; ++i) order[i] = o.order[i];
  return FMMLU_OK;
}

void fmmlu_tree_destroy(fmmlu_tree_h t) { delete t; }

fmmlu_status fmmlu_factor(fmmlu_tree_h t, const double* xyz, const double* normals,
                          const double* weights, double k, double eta, const fmmlu_opts* opts,
                          void* hip_stream, fmmlu_factor_h* out) {
  if (!out) return fail(FMMLU_EINVAL, "out is NULL");
  *out = nullptr;
  return guarded([&] {
    const fmmlu_opts o = checked_opts(t, xyz, normals, weights, k, eta, opts);
    *out = make_factor(t, xyz, normals, weights, k, eta, o, static_cast<hipStream_t>(hip_stream));
  });
}

fmmlu_status fmmlu_factor_batch(int32_t count, const fmmlu_tree_h* trees, const double* const* xyz,
                                const double* const* normals, const double* const* weights, const double* k,
                                const double* eta, const fmmlu_opts* opts, int32_t nthreads, fmmlu_batch_h* out) {
  if (!out) return fail(FMMLU_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(FMMLU_EINVAL, "count must be >= 1");
  if (!trees || !xyz || !normals || !weights || !k || !eta) return fail(FMMLU_EINVAL, "array pointer is NULL");
  return guarded([&] {
    if (opts && opts->corr_row_ptr)
      throw Error(FMMLU_EINVAL, "quadrature corrections are per problem: use fmmlu_factor");
    std::vector<fmmlu_opts> os(count);
    for (int i = 0; i < count; ++i) {
      try {
        os[i] = checked_opts(trees[i], xyz[i], normals[i], weights[i], k[i], eta[i], opts);
      } catch (const Error& e) {
        throw Error(e.status, "problem " + std::to_string(i) + ": " + e.what());
      }
    }
    auto* b = new fmmlu_batch_s;
    try {
      b->factors.assign(count, nullptr);
      int dev = 0;
      FMMLU_HIP(hipGetDevice(&dev));
      const int nt = std::max(1, std::min<int>(count, nthreads > 0 ? nthreads : 8));
      std::atomic<int> next{0};
      std::vector<fmmlu_status> st(count, FMMLU_OK);
      std::vector<std::string> msg(count);
      auto worker = [&]() {
        hipStream_t s = nullptr;
        if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
          (void)hipGetLastError();
          for (int i = next++; i < count; i = next++) {
            st[i] = FMMLU_EHIP;
            msg[i] = "worker stream creation failed";
          }
          return;
        }
        for (int i = next++; i < count; i = next++) {
          try {
            b->factors[i] = make_factor(trees[i], xyz[i], normals[i], weights[i], k[i], eta[i], os[i], s, false);
          } catch (const Error& e) {
            st[i] = e.status;
            msg[i] = e.what();
          } catch (const std::bad_alloc&) {
            st[i] = FMMLU_ENOMEM;
            msg[i] = "host allocation failed";
          } catch (const std::exception& e) {
            st[i] = FMMLU_EHIP;
            msg[i] = e.what();
          }
        }
        (void)hipStreamDestroy(s);
      };
      std::vector<std::thread> pool;
      for (int i = 1; i < nt; ++i) pool.emplace_back(worker);
      worker();
      for (auto& th : pool) th.join();
      for (int i = 0; i < count; ++i)
        if (st[i] != FMMLU_OK) throw Error(st[i], "problem " + std::to_string(i) + ": " + msg[i]);
      b->offsets.assign(count + 1, 0);
      std::vector<FactorImpl*> fs(count);
      for (int i = 0; i < count; ++i) {
        b->offsets[i + 1] = b->offsets[i] + b->factors[i]->f.n;
        fs[i] = &b->factors[i]->f;
      }
      b->solver.init(fs, b->offsets);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

fmmlu_status fmmlu_batch_info(fmmlu_batch_h b, int32_t* count, int64_t* offsets) {
  if (!b) return fail(FMMLU_ESTATE, "batch is NULL");
  if (count) *count = (int32_t)b->factors.size();
  if (offsets) std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  return FMMLU_OK;
}

fmmlu_status fmmlu_batch_factor(fmmlu_batch_h b, int32_t i, fmmlu_factor_h* out) {
  if (!b) return fail(FMMLU_ESTATE, "batch is NULL");
  if (!out) return fail(FMMLU_EINVAL, "out is NULL");
  if (i < 0 || i >= (int32_t)b->factors.size()) return fail(FMMLU_EINVAL, "index out of range");
  *out = b->factors[i];
  return FMMLU_OK;
}

fmmlu_status fmmlu_batch_solve(fmmlu_batch_h b, const void* rhs, void* x, int32_t adjoint, void* hip_stream) {
  if (!b) return fail(FMMLU_ESTATE, "batch is NULL");
  if (!rhs || !x) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  return guarded([&] {
    b->solver.solve(static_cast<const zd*>(rhs), static_cast<zd*>(x), adjoint != 0,
                    static_cast<hipStream_t>(hip_stream));
  });
}

void fmmlu_batch_destroy(fmmlu_batch_h b) { delete b; }

fmmlu_status fmmlu_solve(fmmlu_factor_h f, const void* b, void* x, int64_t nrhs, void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!b || !x) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  if (nrhs < 1) return fail(FMMLU_EINVAL, "nrhs must be >= 1");
  return guarded([&] {
    f->f.solve(static_cast<const zd*>(b), static_cast<zd*>(x), nrhs, false,
               static_cast<hipStream_t>(hip_stream));
  });
}

fmmlu_status fmmlu_set_solve_graph(fmmlu_factor_h f, int32_t enable) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  f->f.use_graph = enable != 0;
  return FMMLU_OK;
}

fmmlu_status fmmlu_solve_adjoint(fmmlu_factor_h f, const void* b, void* x, int64_t nrhs,
                                 void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!b || !x) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  if (nrhs < 1) return fail(FMMLU_EINVAL, "nrhs must be >= 1");
  return guarded([&] {
    f->f.solve(static_cast<const zd*>(b), static_cast<zd*>(x), nrhs, true,
               static_cast<hipStream_t>(hip_stream));
  });
}

fmmlu_status fmmlu_matvec(fmmlu_factor_h f, int32_t op, const void* x, void* y, void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!x || !y) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  if (x == y) return fail(FMMLU_EINVAL, "x and y must not alias");
  if (op < 0 || op > 3) return fail(FMMLU_EINVAL, "op must be 0..3");
  return guarded([&] {
    FactorImpl& F = f->f;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    F.matvec(op, static_cast<const zd*>(x), static_cast<zd*>(y), st);
    FMMLU_HIP(hipStreamSynchronize(st));
  });
}

fmmlu_status fmmlu_matvec_noalloc(fmmlu_factor_h f, int32_t op, const void* x, void* y, void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!x || !y) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  if (x == y) return fail(FMMLU_EINVAL, "x and y must not alias");
  if (op < 0 || op > 3) return fail(FMMLU_EINVAL, "op must be 0..3");
  return guarded([&] {
    FactorImpl& F = f->f;
    const int64_t need = matvec_noalloc_entries(F.n);
    if (need * (int64_t)sizeof(zd) > (int64_t)kNoallocScratchBytes)
      throw Error(FMMLU_EINVAL, "n = " + std::to_string(F.n) + " needs " + std::to_string(need * sizeof(zd)) +
                                    " bytes of matvec scratch; the static scratch holds " +
                                    std::to_string(kNoallocScratchBytes));
    int dev = 0;
    FMMLU_HIP(hipGetDevice(&dev));
    if (dev != F.device)
      throw Error(FMMLU_EINVAL, "the current device (" + std::to_string(dev) + ") is not the factor's device (" +
                                    std::to_string(F.device) + ")");
    zd* ws = noalloc_scratch();
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    zd* xt = ws;
    zd* yt = ws + F.n;
    zd* part = ws + 2 * F.n;
    launch_permute(static_cast<const zd*>(x), xt, F.order_dev, F.n, 1, st);
    launch_matvec(F.g, op, xt, yt, part, matvec_noalloc_part_entries(F.n), st);
    launch_permute(yt, static_cast<zd*>(y), F.order_dev, F.n, 0, st);
  });
}

fmmlu_status fmmlu_farfield(fmmlu_factor_h f, const double* dirs, int64_t ndir, int32_t op, const void* in,
                            void* out, void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!dirs || !in || !out) return fail(FMMLU_EINVAL, "pointer is NULL");
  if (in == out) return fail(FMMLU_EINVAL, "in and out must not alias");
  if (ndir < 1 || ndir > (int64_t(1) << 31) - 1) return fail(FMMLU_EINVAL, "ndir must be in [1, 2^31)");
  if (op < 0 || op > 3) return fail(FMMLU_EINVAL, "op must be 0..3");
  return guarded([&] {
    FactorImpl& F = f->f;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t need = ndir * farfield_chunks(F.n);
    if (op != 1 && need > F.fpart_cap) {
      F.fpart = F.farena.alloc_n<zd>((size_t)need);
      F.fpart_cap = need;
    }
    launch_farfield(F.g, op, dirs, ndir, F.order_dev, static_cast<const zd*>(in), static_cast<zd*>(out), F.fpart,
                    st);
    FMMLU_HIP(hipStreamSynchronize(st));
  });
}

fmmlu_status fmmlu_solve_refined(fmmlu_factor_h f, const void* b, void* x, int32_t adjoint, double tol,
                                 int32_t maxit, int32_t* iters, double* relres, void* hip_stream) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!b || !x) return fail(FMMLU_EINVAL, "vector pointer is NULL");
  if (b == x) return fail(FMMLU_EINVAL, "b and x must not alias");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FMMLU_EINVAL, "tol must be positive");
  if (maxit < 1) return fail(FMMLU_EINVAL, "maxit must be >= 1");
  int32_t it = 0;
  double rr = 0.0;
  fmmlu_status stt = guarded([&] {
    const bool ok = f->f.refine(static_cast<const zd*>(b), static_cast<zd*>(x), adjoint != 0, tol, maxit, &it,
                                &rr, static_cast<hipStream_t>(hip_stream));
    if (!ok)
      throw Error(FMMLU_ENOCONV, "refinement stopped at relative residual " + std::to_string(rr) + " after " +
                                     std::to_string(it) + " iterations");
  });
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return stt;
}

fmmlu_status fmmlu_factor_info(fmmlu_factor_h f, fmmlu_info* out) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  if (!out) return fail(FMMLU_EINVAL, "out is NULL");
  *out = f->f.info;
  return FMMLU_OK;
}

fmmlu_status fmmlu_factor_boxes(fmmlu_factor_h f, int64_t* count, int32_t* level, int32_t* coord,
                                int32_t* m, int32_t* s, int64_t* skel) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  const auto& bx = f->f.boxes;
  if (count) *count = (int64_t)bx.size();
  int64_t pos = 0;
  for (size_t r = 0; r < bx.size(); ++r) {
    if (level) level[r] = bx[r].level;
    if (coord)
      for (int a = 0; a < 3; ++a) coord[3 * r + a] = bx[r].coord[a];
    if (m) m[r] = bx[r].m;
    if (s) s[r] = bx[r].s;
    if (skel)
      for (int64_t v : bx[r].skel_orig) skel[pos++] = v;
  }
  return FMMLU_OK;
}

fmmlu_status fmmlu_factor_box_data(fmmlu_factor_h f, int64_t rec, int32_t* sizes, int64_t* R, int64_t* S,
                                   int64_t* SN, void* T, void* Xi, void* L, void* UT) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  const auto& bx = f->f.boxes;
  if (rec < 0 || rec >= (int64_t)bx.size()) return fail(FMMLU_EINVAL, "record index out of range");
  return guarded([&] {
    const FactorImpl& F = f->f;
    const SolveBox& d = bx[(size_t)rec].dev;
    const int64_t r = d.r, s = d.s, nsn = d.nsn;
    if (sizes) {
      sizes[0] = (int32_t)r;
      sizes[1] = (int32_t)s;
      sizes[2] = (int32_t)nsn;
    }
    int dev = 0;
    FMMLU_HIP(hipGetDevice(&dev));
    if (dev != F.device) FMMLU_HIP(hipSetDevice(F.device));
    FMMLU_HIP(hipDeviceSynchronize());
    auto idx = [&](const int32_t* src, int64_t cnt, int64_t* out) {
      if (!out || cnt == 0) return;
      std::vector<int32_t> h((size_t)cnt);
      FMMLU_HIP(hipMemcpy(h.data(), src, sizeof(int32_t) * (size_t)cnt, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < cnt; ++i) out[i] = F.order[(size_t)h[(size_t)i]];
    };
    auto mat = [&](const void* src, int64_t cnt, void* out) {
      if (!out || cnt == 0) return;
      zd* o = static_cast<zd*>(out);
      if (F.f32) {
        std::vector<zf> h((size_t)cnt);
        FMMLU_HIP(hipMemcpy(h.data(), src, sizeof(zf) * (size_t)cnt, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < cnt; ++i) o[i] = widen(h[(size_t)i]);
      } else {
        FMMLU_HIP(hipMemcpy(o, src, sizeof(zd) * (size_t)cnt, hipMemcpyDeviceToHost));
      }
    };
    idx(d.R, r, R);
    idx(d.S, s, S);
    idx(d.SN, nsn, SN);
    mat(d.T, s * r, T);
    mat(d.Xi, r * r, Xi);
    mat(d.Lp, nsn * r, L);
    mat(d.UpT, nsn * r, UT);
    if (dev != F.device) FMMLU_HIP(hipSetDevice(dev));
  });
}

fmmlu_status fmmlu_factor_profile(fmmlu_factor_h f, double* ms, int64_t* launches, double* flops,
                                  double* bytes) {
  if (!f) return fail(FMMLU_ESTATE, "factor is NULL");
  const Profiler& p = f->f.prof;
  for (int c = 0; c < KC_COUNT; ++c) {
    if (ms) ms[c] = p.ms[c];
    if (launches) launches[c] = p.launches[c];
    if (flops) flops[c] = p.flops[c];
    if (bytes) bytes[c] = p.bytes[c];
  }
  return FMMLU_OK;
}

void fmmlu_factor_destroy(fmmlu_factor_h f) { delete f; }

fmmlu_status fmmlu_dense_inverse(const void* a, int64_t n, int64_t count, void* out, void* hip_stream) {
  if (!a || !out) return fail(FMMLU_EINVAL, "NULL pointer");
  if (a == out) return fail(FMMLU_EINVAL, "a and out must not alias");
  if (n < 1 || n > 65535 || count < 1) return fail(FMMLU_EINVAL, "bad sizes");
  return guarded([&] {
    dense_inverse_batch(static_cast<const zd*>(a), n, count, static_cast<zd*>(out),
                        static_cast<hipStream_t>(hip_stream));
  });
}

namespace {
// SoA geometry with sqrt(w) packed on the device (original order), 7 * n doubles in a
double* pack_geometry(DeviceArena& a, const double* xyz, const double* nrm, const double* w, int64_t n,
                      hipStream_t st) {
  double* p = a.alloc_n<double>(7 * (size_t)n);
  FMMLU_HIP(hipMemcpyAsync(p, xyz, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  FMMLU_HIP(hipMemcpyAsync(p + 3 * n, nrm, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  std::vector<double> hw(n), hs(n);
  FMMLU_HIP(hipMemcpyAsync(hw.data(), w, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  FMMLU_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    if (!(hw[i] > 0.0)) throw Error(FMMLU_EINVAL, "weights must be positive");
    hs[i] = std::sqrt(hw[i]);
  }
  FMMLU_HIP(hipMemcpyAsync(p + 6 * n, hs.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  FMMLU_HIP(hipStreamSynchronize(st));
  return p;
}

// indices must address the geometry: checked on the host before any kernel reads them
void check_indices(const int64_t* dev, int64_t cnt, int64_t n, hipStream_t st, const char* what) {
  std::vector<int64_t> h((size_t)cnt);
  if (cnt) FMMLU_HIP(hipMemcpyAsync(h.data(), dev, sizeof(int64_t) * cnt, hipMemcpyDeviceToHost, st));
  FMMLU_HIP(hipStreamSynchronize(st));
  for (int64_t v : h)
    if (v < 0 || v >= n) throw Error(FMMLU_EINVAL, std::string(what) + " index out of range");
}
}  // namespace

fmmlu_status fmmlu_kernel_block(const double* xyz, const double* nrm, const double* w, int64_t n,
                                double k, double eta, const int64_t* rows, int64_t nr,
                                const int64_t* cols, int64_t nc, void* out, void* hip_stream) {
  if (!xyz || !nrm || !w || !rows || !cols || !out) return fail(FMMLU_EINVAL, "NULL pointer");
  if (n < 1 || nr < 0 || nc < 0) return fail(FMMLU_EINVAL, "bad sizes");
  return guarded([&] {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    DeviceArena a(size_t(8) << 20);
    double* p = pack_geometry(a, xyz, nrm, w, n, st);
    check_indices(rows, nr, n, st, "row");
    check_indices(cols, nc, n, st, "column");
    DevGeom g{p, n, k, eta};
    launch_block(g, rows, nr, cols, nc, static_cast<zd*>(out), st);
    FMMLU_HIP(hipStreamSynchronize(st));
  });
}

fmmlu_status fmmlu_proxy_block(const double* xyz, const double* nrm, const double* w, int64_t n, double k,
                               double eta, const int64_t* dofs, int64_t m, const double* centre, double radius,
                               int32_t ngamma, void* out, void* hip_stream) {
  if (!xyz || !nrm || !w || !dofs || !centre || !out) return fail(FMMLU_EINVAL, "NULL pointer");
  if (n < 1 || m < 1 || m > (int64_t(1) << 30) || ngamma < 1 || ngamma > (1 << 24))
    return fail(FMMLU_EINVAL, "bad sizes");
  if (!(radius > 0.0) || !std::isfinite(radius)) return fail(FMMLU_EINVAL, "radius must be positive");
  return guarded([&] {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    DeviceArena a(size_t(8) << 20);
    double* p = pack_geometry(a, xyz, nrm, w, n, st);
    check_indices(dofs, m, n, st, "dof");
    IdTask t{};
    t.M = static_cast<zd*>(out);
    t.rows = 2 * ngamma;
    t.m = (int32_t)m;
    t.nq = 0;
    t.ngamma = ngamma;
    t.nseg = 0;
    t.seg_off = 0;
    t.dof_off = 0;
    t.cx = centre[0];
    t.cy = centre[1];
    t.cz = centre[2];
    t.radius = radius;
    t.wgamma = std::sqrt(4.0 * M_PI * radius * radius / ngamma);
    t.unit_begin = 0;
    const int64_t units = int64_t((t.rows + 63) / 64) * ((m + 63) / 64);
    IdTask* dt = a.alloc_n<IdTask>(1);
    FMMLU_HIP(hipMemcpyAsync(dt, &t, sizeof(IdTask), hipMemcpyHostToDevice, st));
    DevGeom g{p, n, k, eta};
    launch_build_idmatrix(g, dt, 1, units, nullptr, dofs, nullptr, false, st);
    FMMLU_HIP(hipStreamSynchronize(st));
  });
}

fmmlu_status fmmlu_trim_caches(void) {
  return guarded([&] { trim_reuse_caches(); });
}

fmmlu_status fmmlu_gemm_tuning(char* buf, int64_t len, int64_t* needed) {
  return guarded([&] {
    const std::string r = gemm_tune_report();
    if (r.empty()) throw Error(FMMLU_ESTATE, "no GEMM tuning on this device yet");
    const int64_t need = (int64_t)r.size() + 1;
    if (needed) *needed = need;
    if (buf == nullptr && len == 0) return;
    if (!buf || len < need) throw Error(FMMLU_EINVAL, "buffer too small for the tuning table");
    std::memcpy(buf, r.c_str(), (size_t)need);
  });
}

const char* fmmlu_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
