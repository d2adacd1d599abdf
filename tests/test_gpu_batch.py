"""Batches of independent scatterers: concurrent factorizations on several host threads and
streams, and solves replayed from one graph with a branch per problem. Each problem's
solution is checked against the oracle's dense LU (<= 10 eps), against the same problem
factored alone (identical arithmetic, so identical results), and, for the full 64-scatterer
workload, by the residual on sampled rows formed by the oracle's exact matvec."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import cmatvec, dense

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


def _rhs(s):
    c = np.array([0.1, 0.2, 0.3]) * np.array(s.meta.get("axes", (1.0, 1.0, 1.0)))
    return np.sqrt(s.weights) * synth.point_source_data(s.points, s.k, src=tuple(c))


def test_small_batch_matches_dense_and_single():
    surfs = synth.scatterer_batch(count=6, seed=3, nmin=1200, nmax=3000)
    eps = 1e-5
    say("batch of", [s.n for s in surfs], "k", [round(s.k, 2) for s in surfs])
    batch = fm.FactorBatch([(s.points, s.normals, s.weights, s.k, s.eta) for s in surfs], eps=eps, nthreads=3)
    off = batch.offsets
    b = np.concatenate([_rhs(s) for s in surfs])
    x = batch.solve(torch.as_tensor(b).cuda()).cpu().numpy()
    y = batch.solve(torch.as_tensor(b).cuda(), adjoint=True).cpu().numpy()
    for i, s in enumerate(surfs):
        a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
        bi = b[off[i]:off[i + 1]]
        xs = np.linalg.solve(a, bi)
        ys = np.linalg.solve(a.conj().T, bi)
        ex = np.linalg.norm(x[off[i]:off[i + 1]] - xs) / np.linalg.norm(xs)
        ey = np.linalg.norm(y[off[i]:off[i + 1]] - ys) / np.linalg.norm(ys)
        single = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=eps)
        xi = single.solve(torch.as_tensor(bi).cuda()).cpu().numpy()
        same = np.array_equal(xi, x[off[i]:off[i + 1]])
        say(f"problem {i}: n={s.n} err {ex:.2e} adjoint {ey:.2e}, identical to single factor: {same}")
        assert ex < 10 * eps and ey < 10 * eps
        assert np.abs(xi - x[off[i]:off[i + 1]]).max() <= 1e-13 * np.abs(xi).max()
        # borrowed per-problem handle works and agrees
        fi = batch.factor(i)
        assert fi.info()["n"] == s.n
        r = fi.matvec(torch.as_tensor(x[off[i]:off[i + 1]]).cuda()).cpu().numpy() - bi
        assert np.linalg.norm(r) / np.linalg.norm(bi) < 10 * eps


def test_small_batch_fp32_factors():
    """The same six scatterers with complex float32 factors (the batched workload's stated
    precision): every problem within 10 eps of the oracle's dense LU, forward and adjoint,
    and bitwise equal to the problem factored alone in float32."""
    surfs = synth.scatterer_batch(count=6, seed=3, nmin=1200, nmax=3000)
    eps = 1e-5
    batch = fm.FactorBatch([(s.points, s.normals, s.weights, s.k, s.eta) for s in surfs], eps=eps, nthreads=3,
                           precision=1)
    off = batch.offsets
    b = np.concatenate([_rhs(s) for s in surfs])
    x = batch.solve(torch.as_tensor(b).cuda()).cpu().numpy()
    y = batch.solve(torch.as_tensor(b).cuda(), adjoint=True).cpu().numpy()
    for i, s in enumerate(surfs):
        a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
        bi = b[off[i]:off[i + 1]]
        ex = np.linalg.norm(x[off[i]:off[i + 1]] - np.linalg.solve(a, bi)) / np.linalg.norm(np.linalg.solve(a, bi))
        ys = np.linalg.solve(a.conj().T, bi)
        ey = np.linalg.norm(y[off[i]:off[i + 1]] - ys) / np.linalg.norm(ys)
        single = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=eps, precision=1)
        xi = single.solve(torch.as_tensor(bi).cuda()).cpu().numpy()
        say(f"fp32 problem {i}: n={s.n} err {ex:.2e} adjoint {ey:.2e}")
        assert ex < 10 * eps and ey < 10 * eps
        assert np.abs(xi - x[off[i]:off[i + 1]]).max() <= 1e-13 * np.abs(xi).max()


def test_full_batch_64_scatterers_residual():
    """The 64-scatterer workload (seed 3, sizes 2,000-20,000, k in [1, 8], eps = 1e-5):
    per-problem relative residual on 200 sampled rows, (A~ x - b)[rows], with A~ x formed row
    by row by the oracle's exact matvec."""
    surfs = synth.scatterer_batch()
    eps = 1e-5
    ntot = sum(s.n for s in surfs)
    say(f"64 scatterers, {ntot} unknowns")
    t0 = time.perf_counter()
    batch = fm.FactorBatch([(s.points, s.normals, s.weights, s.k, s.eta) for s in surfs], eps=eps)
    torch.cuda.synchronize()
    say(f"  batch factor {time.perf_counter() - t0:.2f} s")
    b = np.concatenate([_rhs(s) for s in surfs])
    bd = torch.as_tensor(b).cuda()
    x = batch.solve(bd).cpu().numpy()
    rng = np.random.default_rng(0)
    worst = 0.0
    for i, s in enumerate(surfs):
        lo, hi = int(batch.offsets[i]), int(batch.offsets[i + 1])
        rows = np.sort(rng.choice(s.n, 200, replace=False))
        ax = cmatvec.matvec_rows(s.points, s.normals, s.weights, s.k, s.eta, x[lo:hi], rows)
        rel = np.linalg.norm(ax - b[lo:hi][rows]) / np.linalg.norm(b[lo:hi][rows])
        worst = max(worst, float(rel))
    say(f"  worst relative residual on sampled rows (oracle matvec) {worst:.2e}")
    assert worst < 10 * eps
