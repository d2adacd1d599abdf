"""Locally corrected quadrature (Section 5.3) on the GPU, through the C ABI, against the
oracle with the same correction table (synthetic target-dependent weights
w_ij = w_j (1 + a_ij) for near pairs, a few of which reach beyond a box's near field):

* the exact product with all four operators equals the oracle's dense corrected matrices;
* solve and adjoint solve within 10 eps of the oracle's dense LU of the corrected matrix,
  and some owners moved into Q by the spill-over rule;
* Householder route: box by box the oracle's ranks and skeleton sets (schedule
  "phase_start", spill-over on), excluding near-ties and what they change downstream.
"""
import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth
from oracle import dense, rss

pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps / 2


def say(*a):
    print("[corr]", *a, flush=True)


@pytest.fixture(scope="module")
def case():
    s = synth.graded_ellipsoid(2500, seed=2, k=3.0, eps=1e-6)
    corr = synth.near_corrections(s.points, seed=1, long_frac=0.03, long_factor=14.0)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta, corr=corr)
    return s, corr, a


@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_corrected_exact_matvec(case, op):
    s, corr, a = case
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, leaf_size=32, corrections=corr)
    if op == 0:
        m = a
    elif op == 1:
        m = a.conj().T
    else:
        m = dense.derivative_matrix(s.points, s.normals, s.weights, s.k, s.eta, "k" if op == 2 else "eta", corr=corr)
    v = np.random.default_rng(op).standard_normal(s.n) * (1 - 0.5j)
    got = f.matvec(torch.as_tensor(v).cuda(), op).cpu().numpy()
    ref = m @ v
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say("op", op, "rel err", err)
    assert err < 1e-13


@pytest.mark.parametrize("route", [1, 2])
def test_corrected_solves_match_dense(case, route):
    s, corr, a = case
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, leaf_size=32, corrections=corr,
                  id_route=route)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    xs, ys = np.linalg.solve(a, b), np.linalg.solve(a.conj().T, b)
    x = f.solve(torch.as_tensor(b).cuda()).cpu().numpy()
    y = f.solve_adjoint(torch.as_tensor(b).cuda()).cpu().numpy()
    ex = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    ey = np.linalg.norm(y - ys) / np.linalg.norm(ys)
    info = f.info()
    say(f"route {route}: solve {ex:.2e} adjoint {ey:.2e}, spill-over owners {info['nspill']}")
    assert ex <= 10 * s.eps and ey <= 10 * s.eps
    assert info["nspill"] > 0


def test_corrected_householder_matches_oracle_box_by_box(case):
    s, corr, _ = case
    of = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, leaf_size=32, schedule="phase_start",
                       corr=corr)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, leaf_size=32, corrections=corr, id_route=2)
    bx = f.boxes()
    gg = [(int(l), tuple(int(v) for v in c), int(m)) for l, c, m in zip(bx["level"], bx["coord"], bx["m"])]
    assert gg == [(b.level, tuple(b.coord), b.m) for b in of.factors]
    assert f.info()["nspill"] == of.spill_count
    dirty = np.zeros(s.n, bool)
    compared = 0
    pos = 0
    for rec, ob in enumerate(of.factors):
        sk = bx["skel"][pos:pos + bx["s"][rec]]
        pos += bx["s"][rec]
        mg = ob.margins
        if min(mg["gap1"], mg["trunc1"]) <= 1e3 * U * np.sqrt(ob.m) or \
                dirty[np.concatenate([ob.cols, ob.N, ob.Q])].any():
            dirty[np.concatenate([ob.cols, ob.N])] = True
            continue
        assert np.array_equal(sk, np.sort(ob.S)), f"record {rec}: skeleton sets differ"
        compared += 1
    say("records", len(of.factors), "compared", compared, "spill-over owners", of.spill_count)
    assert compared >= 1
