// Iterative refinement with the factored inverse as preconditioner (the use of a direct
// solver as a preconditioner suggested in Section 7): restarted flexible GMRES in float64,
// right-preconditioned, on A~ (or A~^H for the adjoint) applied exactly on the fly.
// Inner products use a fixed partition of the vector and are summed on the host in a
// fixed order, so the iteration is deterministic.
#include <cmath>
#include <complex>
#include <vector>

#include "factor.hpp"

namespace fmmlu {

namespace {

using cd = std::complex<double>;

cd dotc(const zd* x, const zd* y, int64_t n, zd* part, hipStream_t st) {
  launch_dotc_partial(x, y, n, part, st);
  std::vector<zd> h(kDotBlocks);
  FMMLU_HIP(hipMemcpyAsync(h.data(), part, sizeof(zd) * kDotBlocks, hipMemcpyDeviceToHost, st));
  FMMLU_HIP(hipStreamSynchronize(st));
  cd s = 0;
  for (auto& v : h) s += cd(v.re, v.im);
  return s;
}

zd z(cd v) { return zd{v.real(), v.imag()}; }

constexpr int kRestart = 30;  // GMRES restart length

}  // namespace

void FactorImpl::matvec(int op, const zd* x, zd* y, hipStream_t st) {
  ensure_workspace();
  launch_permute(x, wmv, order_dev, n, 1, st);
  launch_matvec(g, op, wmv, ws1.x, wpart, wpart_entries, st);
  launch_permute(ws1.x, y, order_dev, n, 0, st);
}

bool FactorImpl::refine(const zd* b, zd* x, bool adjoint, double tol, int maxit, int* iters_out,
                        double* relres_out, hipStream_t st) {
  ensure_workspace();
  const int m = kRestart;
  const int op = adjoint ? 1 : 0;
  if (!rbuf) rbuf = rarena.alloc_n<zd>((size_t)n * (2 * m + 3) + kDotBlocks);
  zd* V = rbuf;
  zd* Z = V + (size_t)n * (m + 1);
  zd* w = Z + (size_t)n * m;
  zd* r = w + n;
  zd* part = r + n;
  auto precond = [&](const zd* in, zd* out) { solve(in, out, 1, adjoint, st); };
  const double bnorm = std::sqrt(std::abs(dotc(b, b, n, part, st)));
  if (bnorm == 0.0) {
    FMMLU_HIP(hipMemsetAsync(x, 0, sizeof(zd) * n, st));
    FMMLU_HIP(hipStreamSynchronize(st));
    *iters_out = 0;
    *relres_out = 0.0;
    return true;
  }
  // x0 = 0, so r0 = b needs no product with A~; the first Arnoldi step applies the factored
  // inverse to b (what an initial guess x0 = A_f^{-1} b would cost, without its residual)
  FMMLU_HIP(hipMemsetAsync(x, 0, sizeof(zd) * n, st));
  int iters = 0;
  double relres = 1.0;
  bool first = true;
  for (;;) {
    // true residual of the current iterate; the loop ends only here
    double beta;
    if (first) {
      FMMLU_HIP(hipMemcpyAsync(r, b, sizeof(zd) * n, hipMemcpyDeviceToDevice, st));
      beta = bnorm;
      first = false;
    } else {
      matvec(op, x, w, st);
      launch_sub(b, w, r, n, st);
      beta = std::sqrt(std::abs(dotc(r, r, n, part, st)));
    }
    relres = beta / bnorm;
    if (relres <= tol || iters >= maxit) break;
    launch_scal_copy(zd{1.0 / beta, 0.0}, r, V, n, st);
    std::vector<cd> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gvec(m + 1, 0.0);
    gvec[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m && iters < maxit; ++j) {
      zd* vj = V + (size_t)j * n;
      zd* zj = Z + (size_t)j * n;
      precond(vj, zj);
      matvec(op, zj, w, st);
      // modified Gram-Schmidt
      for (int i = 0; i <= j; ++i) {
        const cd h = dotc(V + (size_t)i * n, w, n, part, st);
        H[(size_t)i + (size_t)j * (m + 1)] = h;
        launch_axpy(z(-h), V + (size_t)i * n, w, n, st);
      }
      const double hn = std::sqrt(std::abs(dotc(w, w, n, part, st)));
      H[(size_t)(j + 1) + (size_t)j * (m + 1)] = hn;
      if (hn > 0.0) launch_scal_copy(zd{1.0 / hn, 0.0}, w, V + (size_t)(j + 1) * n, n, st);
      // Givens rotations on column j
      for (int i = 0; i < j; ++i) {
        const cd a = H[(size_t)i + (size_t)j * (m + 1)], c = H[(size_t)(i + 1) + (size_t)j * (m + 1)];
        H[(size_t)i + (size_t)j * (m + 1)] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
        H[(size_t)(i + 1) + (size_t)j * (m + 1)] = -sn[i] * a + cs[i] * c;
      }
      const cd a = H[(size_t)j + (size_t)j * (m + 1)], c = H[(size_t)(j + 1) + (size_t)j * (m + 1)];
      const double den = std::sqrt(std::norm(a) + std::norm(c));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = c / den;
      }
      H[(size_t)j + (size_t)j * (m + 1)] = den;
      H[(size_t)(j + 1) + (size_t)j * (m + 1)] = 0.0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = std::conj(cs[j]) * gvec[j];
      ++iters;
      jdone = j + 1;
      relres = std::abs(gvec[j + 1]) / bnorm;
      if (relres <= tol || hn == 0.0) break;
    }
    // solve the triangular system and update x += Z y
    std::vector<cd> yv(jdone);
    for (int i = jdone - 1; i >= 0; --i) {
      cd sacc = gvec[i];
      for (int l = i + 1; l < jdone; ++l) sacc -= H[(size_t)i + (size_t)l * (m + 1)] * yv[l];
      const cd d = H[(size_t)i + (size_t)i * (m + 1)];
      yv[i] = d == 0.0 ? 0.0 : sacc / d;  // singular Hessenberg: drop the direction
    }
    for (int i = 0; i < jdone; ++i) launch_axpy(z(yv[i]), Z + (size_t)i * n, x, n, st);
  }
  FMMLU_HIP(hipStreamSynchronize(st));
  *iters_out = iters;
  *relres_out = relres;
  return relres <= tol;
}

}  // namespace fmmlu
