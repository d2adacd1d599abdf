"""Far-field pattern operator and adjoint gradients of the far-field loss on the GPU.

The operator is compared entry by entry with the oracle's dense far-field matrix; the
gradients of L = sum_m |F(d_m)|^2 (plane-wave incidence, sigma~ = A~^{-1} b~) with respect
to b~, k and eta are compared with the oracle's dense-LU adjoint gradient, and with
central differences: along a complex direction in b~ (L is quadratic in b~, so the
difference is exact up to solve error) and in k (refactoring at k +- h, refined solves,
truncation O(h^2))."""
import gc
import sys

import numpy as np
import pytest

import synth
from oracle import farfield

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2201_07325_amd")
ag = pytest.importorskip("paper_2201_07325_amd.autograd")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fm.lib()


def _t(a, grad=False):
    if np.ndim(a) == 0:
        t = torch.tensor(float(a), dtype=torch.float64, device="cuda")
    else:
        t = torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return t.requires_grad_(grad) if grad else t


def _factor(s, eps=None, k=None):
    k = s.k if k is None else k
    return fm.Factor(s.points, s.normals, s.weights, k, s.eta, eps=s.eps if eps is None else eps)


@pytest.mark.parametrize("ndir", [1, 64, 300])
def test_farfield_operator_matches_oracle(ndir):
    s = synth.unit_sphere(9000, k=3.0, eta=2.0)
    say(f"farfield operator n=9000 ndir={ndir}")
    f = _factor(s, eps=1e-3)
    dirs = synth.fibonacci_sphere_dirs(ndir)
    rng = np.random.default_rng(ndir)
    v = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    u = rng.standard_normal(ndir) + 1j * rng.standard_normal(ndir)
    C = farfield.operator(dirs, s.points, s.normals, s.weights, s.k, s.eta)
    Ck = farfield.operator_dk(dirs, s.points, s.normals, s.weights, s.k, s.eta)
    Ce = farfield.operator_deta(dirs, s.points, s.normals, s.weights, s.k)
    dd = _t(dirs)
    for op, ref in ((0, C @ v), (2, Ck @ v), (3, Ce @ v)):
        got = f.farfield(dd, _t(v), op).cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"  op {op} max rel err {err:.2e}")
        assert err < 1e-13
    got = f.farfield(dd, _t(u), 1).cpu().numpy()
    ref = C.conj().T @ u
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  op 1 max rel err {err:.2e}")
    assert err < 1e-13


@pytest.fixture(scope="module")
def grad_case():
    s = synth.unit_sphere(2000, k=3.0, eta=2.0, eps=1e-6)
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    dirs = synth.fibonacci_sphere_dirs(64)
    say("dense oracle gradient n=2000")
    ref = farfield.dense_loss_gradients(s.points, s.normals, s.weights, s.k, s.eta, d, dirs)
    f = _factor(s)
    return s, d, dirs, ref, f


def _loss_and_grads(s, f, d, dirs, tol, k=None):
    k = _t(np.float64(s.k if k is None else k), grad=True)
    eta = _t(np.float64(s.eta), grad=True)
    pts, w = _t(s.points), _t(s.weights)
    b = ag.plane_wave_rhs(pts, w, k, d).detach().requires_grad_(True)
    bk = ag.plane_wave_rhs(pts, w, k, d)  # carries the rhs' own k-dependence
    # route the k-dependence of the rhs through bk while keeping grad_b on the leaf b
    bb = b + (bk - bk.detach())
    L, F = ag.far_field_loss(f, bb, k, eta, _t(dirs), refine_tol=tol)
    L.backward()
    return float(L), b.grad.cpu().numpy(), float(k.grad), float(eta.grad)


@pytest.mark.parametrize("tol", [None, 1e-13])
def test_autograd_matches_dense_adjoint_gradient(grad_case, tol):
    s, d, dirs, ref, f = grad_case
    L, gb, gk, ge = _loss_and_grads(s, f, d, dirs, tol)
    eL = abs(L - ref["L"]) / ref["L"]
    eb = np.linalg.norm(gb - ref["grad_b"]) / np.linalg.norm(ref["grad_b"])
    ek = abs(gk - ref["dL_dk"]) / abs(ref["dL_dk"])
    ee = abs(ge - ref["dL_deta"]) / abs(ref["dL_deta"])
    say(f"tol={tol}: L {eL:.2e}, grad_b {eb:.2e}, dL/dk {ek:.2e}, dL/deta {ee:.2e}")
    bar = 10 * s.eps if tol is None else 1e-9
    assert eL < bar and eb < bar and ek < bar and ee < bar


def test_gradient_wrt_rhs_matches_central_difference(grad_case):
    """G1: exact for the quadratic loss; refined solves keep the solve error at 1e-13."""
    s, d, dirs, ref, f = grad_case
    L0, gb, _, _ = _loss_and_grads(s, f, d, dirs, 1e-13)
    rng = np.random.default_rng(11)
    delta = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    delta *= np.linalg.norm(ref["b"]) / np.linalg.norm(delta)
    t = 0.1
    kk, ee = _t(np.float64(s.k)), _t(np.float64(s.eta))

    def loss_at(b):
        return float(ag.far_field_loss(f, _t(b), kk, ee, _t(dirs), refine_tol=1e-13)[0])

    fd = (loss_at(ref["b"] + t * delta) - loss_at(ref["b"] - t * delta)) / (2 * t)
    an = float(np.real(np.vdot(gb, delta)))
    say(f"G1: fd {fd:.10e} adjoint {an:.10e} rel {abs(fd - an) / abs(fd):.2e}")
    assert abs(fd - an) <= 1e-8 * abs(fd)


def _loss_only(s, f, d, dirs, tol, k):
    with torch.no_grad():
        kt = _t(np.float64(k))
        b = ag.plane_wave_rhs(_t(s.points), _t(s.weights), kt, d)
        return float(ag.far_field_loss(f, b, kt, _t(np.float64(s.eta)), _t(dirs), refine_tol=tol)[0])


def _fd_k(s, d, dirs, h, tol=1e-13):
    out = []
    for sgn in (1, -1):
        kk = s.k + sgn * h
        fk = _factor(s, k=kk)
        out.append(_loss_only(s, fk, d, dirs, tol, kk))
        del fk
        gc.collect()
    return (out[0] - out[1]) / (2 * h)


def test_gradient_wrt_k_matches_central_difference(grad_case):
    """G2: dL/dk (rhs, matrix and far-field terms together) vs refactored central difference."""
    s, d, dirs, ref, f = grad_case
    _, _, gk, _ = _loss_and_grads(s, f, d, dirs, 1e-13)
    fd = _fd_k(s, d, dirs, 1e-4 * s.k)
    say(f"G2: fd {fd:.10e} adjoint {gk:.10e} rel {abs(fd - gk) / abs(fd):.2e}")
    assert abs(fd - gk) <= 1e-6 * abs(fd)


def test_gradient_bumpy_sphere_full_size():
    """Bumpy sphere, n = 100,000, k = 5, eps = 1e-6, 64 far-field directions: dL/dk and a
    directional derivative in b~ from the adjoint match central differences to 1e-6."""
    s = synth.bumpy_sphere()
    rng = np.random.default_rng(4)
    d = synth._uniform_sphere(rng, 1)[:, 0]
    dirs = synth.fibonacci_sphere_dirs(64)
    say("bumpy sphere n=100000: factor")
    f = _factor(s)
    torch.cuda.synchronize()
    say("  factor done", {k: v for k, v in f.info().items() if k in ("n0", "factor_bytes", "t_factor")})
    L0, gb, gk, ge = _loss_and_grads(s, f, d, dirs, 1e-12)
    say(f"  L {L0:.6e} dL/dk {gk:.6e} dL/deta {ge:.6e}")
    delta = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    b0 = farfield.plane_wave_rhs(s.points, s.weights, s.k, d)[0]
    delta *= np.linalg.norm(b0) / np.linalg.norm(delta)
    kk, ee = _t(np.float64(s.k)), _t(np.float64(s.eta))

    def loss_at(b):
        return float(ag.far_field_loss(f, _t(b), kk, ee, _t(dirs), refine_tol=1e-12)[0])

    t = 0.1
    fd_b = (loss_at(b0 + t * delta) - loss_at(b0 - t * delta)) / (2 * t)
    an_b = float(np.real(np.vdot(gb, delta)))
    say(f"  G1 rel {abs(fd_b - an_b) / abs(fd_b):.2e}")
    del f
    gc.collect()
    fd_k = _fd_k(s, d, dirs, 1e-4 * s.k, tol=1e-12)
    say(f"  G2 fd {fd_k:.8e} adjoint {gk:.8e} rel {abs(fd_k - gk) / abs(fd_k):.2e}")
    assert abs(fd_b - an_b) <= 1e-6 * abs(fd_b)
    assert abs(fd_k - gk) <= 1e-6 * abs(fd_k)
