"""Exact matvec at a size where the source-slice count comes from the launch model rather than
the one-slice floor (graded ellipsoid, n = 233,001: a ragged last tile of 41 points).

A~ x (Section 3, eq. disc3) is checked on 200 sampled rows against the oracle's row-wise
product, and the adjoint against it through <A~ x, y> = <x, A~^H y> on random vectors."""
import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth
from oracle import cmatvec

pytestmark = pytest.mark.gpu


def test_matvec_sampled_rows_and_adjoint_identity_n233001():
    s = synth.graded_ellipsoid(233_001, seed=7, eps=1e-4)
    print(f"[matvec-large] n {s.n}", flush=True)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    y = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    ax = f.matvec(torch.as_tensor(x).cuda(), 0).cpu().numpy()
    ahy = f.matvec(torch.as_tensor(y).cuda(), 1).cpu().numpy()
    rows = np.sort(rng.choice(s.n, 200, replace=False))
    rows = np.unique(np.concatenate([rows, [0, s.n - 1]]))  # first and last (ragged) tile too
    ref = cmatvec.matvec_rows(s.points, s.normals, s.weights, s.k, s.eta, x, rows)
    err = np.linalg.norm(ax[rows] - ref) / np.linalg.norm(ref)
    lhs, rhs = np.vdot(y, ax), np.vdot(ahy, x)
    dot = abs(lhs - rhs) / (np.linalg.norm(y) * np.linalg.norm(ax))
    print(f"[matvec-large] sampled rows rel err {err:.2e}, adjoint identity {dot:.2e}", flush=True)
    assert err <= 1e-13
    assert dot <= 1e-13
