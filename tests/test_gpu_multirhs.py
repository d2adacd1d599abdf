"""Blocked multi-right-hand-side solves (blocks of 32 columns through the matrix-core sweeps)
against the single-column sweeps (same factors, different summation order: within 1e-11
relative per column), run-to-run bitwise identical, forward and adjoint, graph and eager
paths, float64 and float32 factors, block sizes below, at and above the block width; plus
the residual of the blocked solution with the exact float64 matvec and the oracle's dense LU."""
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


def _cols(f, B, adjoint):
    fn = f.solve_adjoint if adjoint else f.solve
    return torch.stack([fn(B[:, c].contiguous()) for c in range(B.shape[1])], dim=1)


@pytest.mark.parametrize("precision", [0, 1])
def test_blocked_solves_match_single_columns(precision):
    s = synth.graded_ellipsoid(6000, seed=2)
    eps = 1e-6
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=eps, leaf_size=32, precision=precision)
    rng = np.random.default_rng(7)
    for nrhs in (2, 32, 33, 70):
        B = torch.as_tensor(rng.standard_normal((s.n, nrhs)) + 1j * rng.standard_normal((s.n, nrhs))).cuda()
        for graph in (True, False):
            f.set_solve_graph(graph)
            for adjoint in (False, True):
                X = f.solve_adjoint(B) if adjoint else f.solve(B)
                X2 = f.solve_adjoint(B) if adjoint else f.solve(B)
                ref = _cols(f, B, adjoint)
                torch.cuda.synchronize()
                rel = float((torch.linalg.norm(X - ref, dim=0) / torch.linalg.norm(ref, dim=0)).max())
                say(f"precision {precision} nrhs {nrhs} graph {graph} adjoint {adjoint}: "
                    f"vs single columns {rel:.2e}, repeat equal {torch.equal(X, X2)}")
                assert torch.equal(X, X2)
                assert rel < 1e-11
    f.set_solve_graph(True)
    # residual of a blocked forward solve, column by column, with the exact matvec
    B = torch.as_tensor(rng.standard_normal((s.n, 9)) + 1j * rng.standard_normal((s.n, 9))).cuda()
    X = f.solve(B)
    worst = 0.0
    for c in range(9):
        r = f.matvec(X[:, c].contiguous()) - B[:, c]
        worst = max(worst, float(torch.linalg.norm(r) / torch.linalg.norm(B[:, c])))
    say(f"precision {precision}: worst relative residual of 9 blocked columns {worst:.2e}")
    assert worst < (10 * eps if precision == 0 else 1e-3)


def test_blocked_solves_match_oracle_dense_lu():
    """Thirty-five columns (a block of 32 and a ragged block of three), forward and adjoint,
    against the oracle's dense LU column by column (<= 10 eps)."""
    s = synth.unit_sphere(3000)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    lu = dense.DenseLU(a)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((s.n, 35)) + 1j * rng.standard_normal((s.n, 35))
    B[:, 0] = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    Bd = torch.as_tensor(B).cuda()
    for adjoint in (False, True):
        X = (f.solve_adjoint(Bd) if adjoint else f.solve(Bd)).cpu().numpy()
        ref = lu.solve_adjoint(B) if adjoint else lu.solve(B)
        errs = np.linalg.norm(X - ref, axis=0) / np.linalg.norm(ref, axis=0)
        say(f"adjoint {adjoint}: worst column error vs dense LU {errs.max():.2e}")
        assert errs.max() <= 10 * s.eps


def test_blocked_solve_in_place_and_zero_columns():
    s = synth.graded_ellipsoid(3000, seed=5)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, leaf_size=32)
    rng = np.random.default_rng(3)
    B = torch.as_tensor(rng.standard_normal((s.n, 5)) + 1j * rng.standard_normal((s.n, 5))).cuda()
    B[:, 2] = 0
    ref = f.solve(B)
    torch.cuda.synchronize()
    assert torch.count_nonzero(ref[:, 2]) == 0
    # column-major n x 5 in one buffer, solved in place through the C entry point
    bcol = B.t().contiguous()
    out = fm.lib().fmmlu_solve(f.h, fm.P(bcol.data_ptr()), fm.P(bcol.data_ptr()), 5, fm._stream())
    torch.cuda.synchronize()
    assert out == 0 and torch.equal(bcol.t(), ref)
