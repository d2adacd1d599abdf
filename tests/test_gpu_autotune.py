"""The GEMM autotuner: after a factorization the device's table names, for every use of the
batched GEMM (precision, mapped output, op(A)) and K bucket, one of its candidate kernels
with a measured time for each; and every kernel variant the tuner can choose gives a
factorization that solves to the oracle's dense LU within 10 eps (both precisions), with the
variants' solutions agreeing within the tolerance (float64 factors: a rounding-level change
can move a near-tie pivot of an ID) or the refinement bound (float32 factors)."""
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


def test_tuning_table():
    s = synth.unit_sphere(1500)
    fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, leaf_size=32)
    tab = fm.gemm_tuning()
    assert tab is not None
    ch = tab["choices"]
    say(f"{len(ch)} entries; e.g. {ch[0]}")
    uses = {(c["precision"], c["mapped"], c["opA"]) for c in ch}
    assert uses == {("c128", 1, 0), ("c128", 0, 0), ("c128", 0, 1), ("c128", 0, 2), ("c64", 1, 0), ("c64", 0, 0)}
    for c in ch:
        assert c["k_bucket"] in ("<=32", "<=512", ">512")
        assert c["kernel"] in c["ms"]
        assert all(v > 0 for v in c["ms"].values())
        assert set(c["ms"]) == {"lds64x8", "reg64x8", "reg64x4"}


@pytest.mark.parametrize("precision", [0, 1])
def test_every_kernel_variant_solves(precision):
    s = synth.graded_ellipsoid(2500, seed=3)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    xs = np.linalg.solve(a, b)
    eps = 1e-6
    sols = []
    for mode in (2, 3, 4):
        f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=eps, leaf_size=32, precision=precision,
                      gemm_autotune=mode)
        if precision == 0:
            x = f.solve(torch.as_tensor(b).cuda()).cpu().numpy()
            tol = 10 * eps
        else:
            x, it, rel = f.solve_refined(torch.as_tensor(b).cuda(), tol=1e-10, maxit=30)
            x = x.cpu().numpy()
            tol = 1e-9
        err = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
        say(f"precision {precision} kernel mode {mode}: error vs dense LU {err:.2e}")
        assert err <= tol
        sols.append(x)
    for x in sols[1:]:
        d = float(np.linalg.norm(x - sols[0]) / np.linalg.norm(sols[0]))
        say(f"precision {precision}: variants differ by {d:.2e}")
        assert d <= (20 * eps if precision == 0 else 1e-9)
