"""Float64 refinement of the factored inverse (Section 7: the direct solver used as a
preconditioner): FGMRES with the exact matvec reaches the requested residual, and its
solution agrees with the oracle's dense LU solve of the same system to the conditioning
of the system times the tolerance."""
import sys

import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2201_07325_amd")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fm.lib()


@pytest.fixture(scope="module")
def case():
    s = synth.unit_sphere(2500)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    lu = dense.DenseLU(a)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    say("factor sphere n=2500 eps=1e-3")
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-3)
    torch.cuda.synchronize()
    return s, a, lu, b, f


def test_refined_forward_reaches_tolerance(case):
    s, a, lu, b, f = case
    x0 = f.solve(torch.as_tensor(b).cuda()).cpu().numpy()
    e0 = np.linalg.norm(a @ x0 - b) / np.linalg.norm(b)
    x, it, rr = f.solve_refined(torch.as_tensor(b).cuda(), tol=1e-12, maxit=60)
    x = x.cpu().numpy()
    rr_host = np.linalg.norm(a @ x - b) / np.linalg.norm(b)
    xs = lu.solve(b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    say(f"forward: unrefined relres {e0:.2e}; refined relres {rr:.2e} (host {rr_host:.2e}) in {it} its; "
        f"err vs dense {err:.2e}")
    assert e0 > 1e-6          # the loose factorization alone is far from the tolerance
    assert rr <= 1e-12 and rr_host <= 2e-12
    assert it <= 30
    assert err < 1e-10


def test_refined_adjoint_reaches_tolerance(case):
    s, a, lu, b, f = case
    x, it, rr = f.solve_refined(torch.as_tensor(b).cuda(), adjoint=True, tol=1e-12, maxit=60)
    x = x.cpu().numpy()
    rr_host = np.linalg.norm(a.conj().T @ x - b) / np.linalg.norm(b)
    xs = np.linalg.solve(a.conj().T, b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    say(f"adjoint: refined relres {rr:.2e} (host {rr_host:.2e}) in {it} its; err vs dense {err:.2e}")
    assert rr <= 1e-12 and rr_host <= 2e-12
    assert err < 1e-10


def test_refined_restart_and_noconv(case):
    s, a, lu, b, f = case
    bd = torch.as_tensor(b).cuda()
    # one iteration cannot reach 1e-15 from a 1e-3 factorization
    with pytest.raises(fm.FmmluError) as ei:
        f.solve_refined(bd, tol=1e-15, maxit=1)
    assert ei.value.status == fm.ENOCONV
    x, it, rr = f.solve_refined(bd, tol=1e-15, maxit=1, raise_on_fail=False)
    assert it == 1 and 0 < rr < 1
    rr_host = np.linalg.norm(a @ x.cpu().numpy() - b) / np.linalg.norm(b)
    assert abs(rr_host - rr) <= 1e-3 * rr
    # more iterations than one restart cycle (30) still converge monotonically
    x, it2, rr2 = f.solve_refined(bd, tol=1e-14, maxit=80, raise_on_fail=False)
    assert rr2 < rr


def test_refined_zero_rhs_and_bad_args(case):
    s, a, lu, b, f = case
    z = torch.zeros(s.n, dtype=torch.complex128, device="cuda")
    x, it, rr = f.solve_refined(z)
    assert it == 0 and rr == 0.0 and float(x.abs().max()) == 0.0
    bd = torch.as_tensor(b).cuda()
    for kw in ({"tol": 0.0}, {"tol": -1.0}, {"maxit": 0}):
        with pytest.raises(fm.FmmluError):
            f.solve_refined(bd, **kw)


@pytest.mark.parametrize("leaf", [64, 32])
def test_float32_factors_refined_to_float64_accuracy(leaf):
    """Complex float32 tiles, panels and Schur updates (ID pivoting and pivot-block inverses
    in float64): the factored inverse alone is float32-accurate; float64 FGMRES with the
    exact matvec brings the solution to the dense LU answer."""
    s = synth.unit_sphere(3000)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    xs = dense.DenseLU(a).solve(b)
    f64 = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, leaf_size=leaf)
    f32 = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, leaf_size=leaf, precision=1)
    i32, i64 = f32.info(), f64.info()
    assert i32["precision"] == 1
    bd = torch.as_tensor(b).cuda()
    x32 = f32.solve(bd).cpu().numpy()
    e32 = np.linalg.norm(x32 - xs) / np.linalg.norm(xs)
    y32 = f32.solve_adjoint(bd).cpu().numpy()
    ys = np.linalg.solve(a.conj().T, b)
    ey32 = np.linalg.norm(y32 - ys) / np.linalg.norm(ys)
    x, it, rr = f32.solve_refined(bd, tol=1e-12, maxit=40)
    er = np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs)
    say(f"leaf {leaf}: factor bytes fp32 {i32['factor_bytes']} vs fp64 {i64['factor_bytes']}; "
        f"fp32 solve err {e32:.2e} adjoint {ey32:.2e}; refined {it} its relres {rr:.2e} err {er:.2e}")
    # the top block stays float64 (its dense inverse); every other factor byte halves
    box32 = i32["factor_bytes"] - 16 * i32["n0"] ** 2
    box64 = i64["factor_bytes"] - 16 * i64["n0"] ** 2
    assert box32 < 0.6 * box64
    assert e32 < 1e-4 and ey32 < 1e-4
    assert rr <= 1e-12 and er < 1e-10
