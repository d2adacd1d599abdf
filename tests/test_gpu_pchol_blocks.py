"""The blocked pivoted Cholesky of the Gram route (greedy CPQR, Section 4.1) launches blocks of
pivots up to a bound taken from the ranks seen so far and the remaining blocks only for a
phase whose pivoting had not stopped by then. Forcing one block before the first rank
read-back (fmmlu_opts.pchol_blocks = 1) takes that second path on every wide phase; the
blocks run in the same sequence either way, so ranks, pivots and solutions are identical."""
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


@pytest.mark.parametrize("precision", [0, 1])
def test_forced_continuation_gives_identical_factors(precision):
    # 16,000 points, leaf 64: the upper levels' boxes have well over 128 active DOFs, so
    # their phases take the blocked pivoting
    s = synth.graded_ellipsoid(16000, seed=2)
    b = torch.as_tensor(np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)).cuda()
    out = {}
    for blocks in (0, 1, 3):
        say("graded ellipsoid n=16000, precision", precision, "pchol_blocks", blocks)
        f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, precision=precision,
                      pchol_blocks=blocks)
        bx = f.boxes()
        x = f.solve(b)
        y = f.solve_adjoint(b)
        torch.cuda.synchronize()
        out[blocks] = (bx["s"].copy(), bx["skel"].copy(), x.cpu().numpy(), y.cpu().numpy(),
                       f.info()["max_block"])
        del f
    assert out[0][4] >= 128, "no phase took the blocked pivoting"
    for blocks in (1, 3):
        assert np.array_equal(out[blocks][0], out[0][0])
        assert np.array_equal(out[blocks][1], out[0][1])
        assert np.array_equal(out[blocks][2], out[0][2])
        assert np.array_equal(out[blocks][3], out[0][3])
