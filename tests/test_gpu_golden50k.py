"""The graded-ellipsoid workload at full size (n = 50,000) against the oracle's reference
solutions, element by element.

tests/golden/ellipsoid50k_reference.npz holds x* = A~^{-1} b and y* = A~^{-H} b, written by
tests/golden/make_ellipsoid50k_reference.py with the oracle's float64 GMRES and exact matvec
to a relative residual <= 1e-13 (dense LU of the 40 GB matrix replaced by that iteration).
Bars: the eps-accurate factored inverse within 10 eps in the relative 2-norm of the scaled
unknowns (the bar Section 4.2's eps-accurate factorization is held to), and entry by entry
within 10 eps of max|x*|; refined solves (float64 FGMRES with the exact matvec) within 1e-9.
The blocked sweeps (32 columns on the matrix cores) are held to the same bar on a column
that is b, and to 1e-11 of the single-column solve.
"""
import os

import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ellipsoid50k_reference.npz")


@pytest.fixture(scope="module")
def workload():
    ref = np.load(GOLDEN)
    s = synth.graded_ellipsoid(int(ref["n"]), seed=int(ref["seed"]))
    assert abs(s.k - float(ref["k"])) == 0 and abs(s.eta - float(ref["eta"])) == 0
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k, src=tuple(ref["source"]))
    return s, torch.as_tensor(b).cuda(), ref["x"], ref["y"]


def _errs(x, xs):
    x = x.cpu().numpy()
    return (float(np.linalg.norm(x - xs) / np.linalg.norm(xs)),
            float(np.max(np.abs(x - xs)) / np.max(np.abs(xs))))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_solves_match_oracle_reference(workload, precision):
    s, bd, xs, ys = workload
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, precision=precision)
    bar = 10 * s.eps
    if precision == 0:
        x1, y1 = f.solve(bd), f.solve_adjoint(bd)
        e2, emax = _errs(x1, xs)
        print(f"fp64 solve: rel 2-norm {e2:.2e}, max {emax:.2e}")
        assert e2 <= bar and emax <= bar
        e2, emax = _errs(y1, ys)
        print(f"fp64 adjoint: rel 2-norm {e2:.2e}, max {emax:.2e}")
        assert e2 <= bar and emax <= bar
        # a block of 32 columns through the blocked sweeps (at this size their backward x_R
        # partials are summed once per phase on the upper levels, and the phases with few
        # boxes take items of 16): column 0 is b
        g = torch.Generator().manual_seed(11)
        B = torch.complex(torch.randn(s.n, 32, generator=g, dtype=torch.float64),
                          torch.randn(s.n, 32, generator=g, dtype=torch.float64)).cuda()
        B[:, 0] = bd
        for adj, ref, single in ((False, xs, x1), (True, ys, y1)):
            X = f.solve_adjoint(B) if adj else f.solve(B)
            e2, emax = _errs(X[:, 0], ref)
            d = float(torch.linalg.norm(X[:, 0] - single) / torch.linalg.norm(single))
            print(f"fp64 block of 32 (adjoint={adj}): column 0 rel 2-norm {e2:.2e}, max {emax:.2e}, "
                  f"vs the single-column solve {d:.1e}")
            assert e2 <= bar and emax <= bar and d <= 1e-11
    for adj, ref in ((False, xs), (True, ys)):
        x, its, rel = f.solve_refined(bd, adjoint=adj, tol=1e-12, maxit=60)
        e2, emax = _errs(x, ref)
        print(f"precision {precision} refined (adjoint={adj}): {its} iterations, relres {rel:.1e}, "
              f"rel 2-norm {e2:.2e}, max {emax:.2e}")
        assert rel <= 1e-12 and e2 <= 1e-9 and emax <= 1e-9
