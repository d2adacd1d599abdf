"""Solves replayed from captured HIP graphs give exactly the eager result (same kernels in
the same order), on every replay, with unrelated eager work and synchronisations between
replays; forward and adjoint; several right-hand sides."""
import sys

import numpy as np
import pytest

import synth

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


def test_graph_replays_match_eager():
    s = synth.graded_ellipsoid(6000, seed=2)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-5, leaf_size=32)
    rng = np.random.default_rng(0)
    b = torch.as_tensor(rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)).cuda()
    b2 = torch.as_tensor(rng.standard_normal((s.n, 3)) + 1j * rng.standard_normal((s.n, 3))).cuda()
    f.set_solve_graph(False)
    xe, ye, x2e = f.solve(b), f.solve_adjoint(b), f.solve(b2)
    torch.cuda.synchronize()
    f.set_solve_graph(True)
    for rep in range(5):
        xg = f.solve(b)
        _ = f.matvec(b, 0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        yg = f.solve_adjoint(b)
        x2g = f.solve(b2)
        torch.cuda.synchronize()
        say(f"replay {rep}: fwd equal {torch.equal(xg, xe)}, adj equal {torch.equal(yg, ye)}, "
            f"3 rhs equal {torch.equal(x2g, x2e)}")
        assert torch.equal(xg, xe) and torch.equal(yg, ye) and torch.equal(x2g, x2e)
    # in place (b and x alias) through the graph path
    bb = b.clone()
    out = fm.lib().fmmlu_solve(f.h, fm.P(bb.data_ptr()), fm.P(bb.data_ptr()), 1, fm._stream())
    torch.cuda.synchronize()
    assert out == 0 and torch.equal(bb, xe)
