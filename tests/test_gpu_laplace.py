"""Laplace limit k = 0 through the same code: the combined-field operator D - i eta S with the
static Green's function 1 / (4 pi r). Unit sphere (3,000 Fibonacci points): factored solve
and adjoint solve against dense LU of the oracle's matrix (<= 10 eps), exact matvec against
the dense product, and the float32-factor route refined to 1e-10."""
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


def test_laplace_combined_field_matches_dense():
    s = synth.unit_sphere(3000, k=0.0, eta=1.0, eps=1e-6)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    lu = dense.DenseLU(a)
    rng = np.random.default_rng(11)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, 0.0)
    c = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps)
    x = f.solve(torch.as_tensor(b).cuda()).cpu().numpy()
    xs = lu.solve(b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    xa = f.solve_adjoint(torch.as_tensor(c).cuda()).cpu().numpy()
    xas = lu.solve_adjoint(c)
    erra = np.linalg.norm(xa - xas) / np.linalg.norm(xas)
    y = f.matvec(torch.as_tensor(c).cuda()).cpu().numpy()
    errm = np.linalg.norm(y - a @ c) / np.linalg.norm(a @ c)
    say(f"k = 0: solve {err:.2e}, adjoint {erra:.2e}, matvec {errm:.2e}, info {f.info()}")
    assert err <= 10 * s.eps and erra <= 10 * s.eps and errm <= 1e-13


def test_laplace_float32_refined():
    s = synth.unit_sphere(3000, k=0.0, eta=1.0, eps=1e-6)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, precision=1)
    b = torch.as_tensor(np.sqrt(s.weights) * synth.point_source_data(s.points, 0.0)).cuda()
    x, it, rr = f.solve_refined(b, tol=1e-10, maxit=30)
    r = f.matvec(x) - b
    rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    say(f"k = 0 float32 factors: {it} iterations, relres {rr:.2e} (exact {rel:.2e})")
    assert rel <= 1e-10
