"""The batched dense inverse (blocked Gauss-Jordan with partial pivoting) that inverts the
pivot blocks X_RR and the top block, against LAPACK's inverse on random complex matrices.
Sizes cover every code path: one workgroup per matrix (n <= 320, one to five rows per
lane), the multi-launch pipeline with a single-workgroup panel, and the cooperative panel
(n > 256 rows split over workgroups), and above 2048 rows the panel pipeline whose updates
run as GEMMs on the matrix cores with the shifted identity folded into the A operand; ragged
panel tails; matrices that need row exchanges at every step; an exactly singular matrix."""
import sys

import numpy as np
import pytest

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


def _rand(rng, cnt, n):
    return (rng.standard_normal((cnt, n, n)) + 1j * rng.standard_normal((cnt, n, n))) / np.sqrt(n)


@pytest.mark.parametrize("n,cnt", [(1, 3), (7, 3), (16, 2), (17, 3), (63, 2), (64, 2), (65, 2), (100, 3),
                                   (128, 2), (129, 2), (193, 2), (256, 2), (257, 2), (300, 2), (320, 2),
                                   (321, 2), (513, 1), (1000, 1), (2049, 1), (2600, 1)])
def test_inverse_matches_lapack(n, cnt):
    rng = np.random.default_rng(n)
    a = _rand(rng, cnt, n)
    say(f"dense inverse n={n} count={cnt}")
    x = fm.dense_inverse(torch.as_tensor(a).cuda()).cpu().numpy()
    for i in range(cnt):
        ref = np.linalg.inv(a[i])
        err = np.linalg.norm(x[i] - ref) / np.linalg.norm(ref)
        res = np.linalg.norm(a[i] @ x[i] - np.eye(n)) / np.sqrt(n)
        cond = np.linalg.cond(a[i])
        say(f"  [{i}] rel err {err:.2e} residual {res:.2e} cond {cond:.1e}")
        assert err <= 1e-14 * cond * max(8.0, np.sqrt(n))
        assert res <= 1e-13 * cond


@pytest.mark.parametrize("n", [50, 300, 700])
def test_inverse_needs_row_exchanges(n):
    """A permuted diagonally dominant matrix: every column's pivot sits away from the
    diagonal, so every step exchanges rows."""
    rng = np.random.default_rng(7)
    d = np.diag(4.0 + rng.random(n)) + 0.1 * _rand(rng, 1, n)[0]
    perm = rng.permutation(n)
    a = d[perm]
    x = fm.dense_inverse(torch.as_tensor(a).cuda()).cpu().numpy()
    res = np.linalg.norm(a @ x - np.eye(n)) / np.sqrt(n)
    say(f"row exchanges n={n}: residual {res:.2e}")
    assert res < 1e-13


def test_singular_is_reported():
    a = _rand(np.random.default_rng(3), 1, 40)
    a[0][:, 5] = 0.0
    with pytest.raises(fm.FmmluError) as ei:
        fm.dense_inverse(torch.as_tensor(a).cuda())
    assert ei.value.code == "ESINGULAR"
