"""Per-box parity of the factorization with the oracle, through the C ABI.

The GPU runs each colour phase of a level as one concurrent step: every box of the phase
classifies the DOFs that were active when the phase began. The oracle's
schedule="phase_start" takes the same reading (a box's Q rows then also hold the redundant
DOFs of an earlier same-colour box; those rows lie, to the ID tolerance, in the span of that
box's skeleton rows, so the ID stays valid), so the two compute the same factorization.

Householder route (opts.id_route = 2: blocked Householder QR of the ID matrix, then greedy
column pivoting on R): the pivot decisions are taken on column norms accurate to a few ulps
of the matrix norm, like the oracle's. Every box whose decisions are not near-ties at that
precision (and whose inputs no earlier excluded box has changed) must have the oracle's rank
and skeleton set exactly, and T, X_RR^{-1}, L and U within bounds derived from the
conditioning of the ID and of X_RR.

Gram route (id_route = 1, the default at eps >= 1e-7): greedy pivoting on the Gram matrix
M^H M decides on squared norms accurate only to about u ||M||^2, coarser than the spacing of
the tail pivots, so its skeleton sets are a different valid choice. Each box whose inputs are
the oracle's (no earlier divergence reaches them) is checked for validity instead: its
skeleton and T applied to the oracle's ID matrix give an eps-accurate ID.
"""
import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth
from oracle import rss

pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps / 2

CASES = {
    "sphere3000": (lambda: synth.unit_sphere(3000), 64),
    "ellipsoid2500": (lambda: synth.graded_ellipsoid(2500, seed=2, k=3.0, eps=1e-6), 32),
}


def say(*a):
    print("[perbox]", *a, flush=True)


_ORACLES = {}


def _case(case):
    if case not in _ORACLES:
        make, leaf = CASES[case]
        s = make()
        say(case, "oracle rs-s, phase-start schedule (cpu)")
        _ORACLES[case] = (s, leaf, rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps,
                                                 leaf_size=leaf, schedule="phase_start", keep_id=True))
    return _ORACLES[case]


def _reads(f):
    return np.concatenate([f.cols, f.N, f.Q])


def _perm_to(sorted_ref, idx):
    """positions p with idx[p] == sorted_ref (both hold the same set)."""
    o = np.argsort(idx)
    assert np.array_equal(idx[o], sorted_ref)
    return o


@pytest.mark.parametrize("case", list(CASES))
def test_householder_route_matches_oracle_box_by_box(case):
    s, leaf, of = _case(case)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, leaf_size=leaf, id_route=2)
    bx = f.boxes()
    gg = [(int(l), tuple(int(v) for v in c), int(m)) for l, c, m in zip(bx["level"], bx["coord"], bx["m"])]
    og = [(b.level, tuple(b.coord), b.m) for b in of.factors]
    assert gg == og, "different boxes eliminated, or in a different order"
    dirty = np.zeros(s.n, bool)
    compared = flagged = 0
    worst = {"T": 0.0, "Xi": 0.0, "L": 0.0, "U": 0.0}
    worst_rel = dict(worst)
    for rec, ob in enumerate(of.factors):
        mg = ob.margins
        near_tie = min(mg["gap1"], mg["trunc1"]) <= 1e3 * U * np.sqrt(ob.m)
        if near_tie or dirty[_reads(ob)].any():
            flagged += 1
            dirty[np.concatenate([ob.cols, ob.N])] = True
            continue
        g = f.box_data(rec)
        assert g["S"].size == ob.S.size, f"record {rec}: rank {g['S'].size} vs oracle {ob.S.size}"
        assert np.array_equal(np.sort(g["S"]), np.sort(ob.S)), f"record {rec}: skeleton sets differ"
        compared += 1
        if ob.R.size == 0:
            continue
        # common ordering: S, R and S u N sorted by DOF index
        Ss, Rs = np.sort(ob.S), np.sort(ob.R)
        ps_o, pr_o = _perm_to(Ss, ob.S), _perm_to(Rs, ob.R)
        ps_g, pr_g = _perm_to(Ss, g["S"]), _perm_to(Rs, g["R"])
        SNo = np.concatenate([ob.S, ob.N])
        SNs = np.sort(SNo)
        psn_o, psn_g = _perm_to(SNs, SNo), _perm_to(SNs, g["SN"])
        To, Tg = ob.T[np.ix_(ps_o, pr_o)], g["T"][np.ix_(ps_g, pr_g)]
        Xio = np.linalg.inv(ob.XRR)[np.ix_(pr_o, pr_o)]
        Xig = g["Xi"][np.ix_(pr_g, pr_g)]
        Lo, Lg = ob.Lp[np.ix_(psn_o, pr_o)], g["L"][np.ix_(psn_g, pr_g)]
        Uo, Ug = ob.Up[np.ix_(pr_o, psn_o)], g["U"][np.ix_(pr_g, psn_g)]
        # backward-stable QR: relative error of T <= c u kappa(M_S) (1 + ||T||), c ~ sqrt(m)
        # for the normwise backward error; X_RR, L, U inherit it through products with T and
        # the inversion (kappa(X_RR))
        pos = {int(v): i for i, v in enumerate(ob.cols)}
        ms = ob.M[:, [pos[int(v)] for v in Ss]]
        kap_s = np.linalg.cond(ms)
        kap_x = np.linalg.cond(ob.XRR)
        tn = np.linalg.norm(To, 2)
        c = 10 * np.sqrt(ob.m)
        eT = c * U * kap_s * (1 + tn)
        eX = eT * (1 + tn) * kap_x + c * U * kap_x
        for name, go, oo, bound in (("T", Tg, To, eT), ("Xi", Xig, Xio, eX), ("L", Lg, Lo, eX),
                                    ("U", Ug, Uo, eX)):
            rel = np.linalg.norm(go - oo) / max(np.linalg.norm(oo), 1e-300)
            worst[name] = max(worst[name], rel / bound)
            worst_rel[name] = max(worst_rel[name], rel)
            assert rel <= bound, f"record {rec} {name}: rel err {rel:.2e} > bound {bound:.2e}"
    say(case, "records", len(og), "compared", compared, "excluded (near-tie or downstream)", flagged,
        "worst rel err", {k: f"{v:.1e}" for k, v in worst_rel.items()},
        "worst err/bound", {k: f"{v:.1e}" for k, v in worst.items()})
    assert compared >= 1 and compared + flagged == len(og)


@pytest.mark.parametrize("case", list(CASES))
def test_gram_route_ids_valid_on_oracle_matrices(case):
    s, leaf, of = _case(case)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=s.eps, leaf_size=leaf, id_route=1)
    bx = f.boxes()
    assert len(bx["m"]) == len(of.factors)
    dirty = np.zeros(s.n, bool)
    checked = same = 0
    worst = 0.0
    for rec, ob in enumerate(of.factors):
        g = f.box_data(rec)
        gcols = np.sort(np.concatenate([g["S"], g["R"]]))
        if dirty[_reads(ob)].any() or not np.array_equal(gcols, np.sort(ob.cols)):
            dirty[np.concatenate([ob.cols, ob.N])] = True
            continue
        pos = {int(v): i for i, v in enumerate(ob.cols)}
        cs = np.array([pos[int(v)] for v in g["S"]], np.int64)
        cr = np.array([pos[int(v)] for v in g["R"]], np.int64)
        M = ob.M
        err = np.linalg.norm(M[:, cr] - M[:, cs] @ g["T"], 2) if cr.size else 0.0
        bound = 2 * np.sqrt(cr.size + 1) * s.eps * np.linalg.norm(M, 2)
        worst = max(worst, err / bound)
        assert err <= bound, f"record {rec}: ID error {err:.2e} > {bound:.2e}"
        checked += 1
        if np.array_equal(np.sort(g["S"]), np.sort(ob.S)):
            same += 1
        else:
            dirty[np.concatenate([ob.cols, ob.N])] = True
    say(case, "gram route: records", len(of.factors), "checked", checked, "same skeleton set", same,
        f"worst err/bound {worst:.2f}")
    assert checked >= 1


def test_proxy_rows_match_oracle():
    s = synth.graded_ellipsoid(2000, seed=2, k=3.0)
    t = fm.Tree(s.points, 32).export()
    rng = np.random.default_rng(5)
    # a box at level 3 and one at the finest level, with the DOFs they hold
    x = s.points
    lo, hi = x.min(axis=1), x.max(axis=1)
    side0 = (hi - lo).max() * (1 + 1e-12)
    c0 = 0.5 * (lo + hi)
    for lev in (3, int(t["level"].max())):
        side = side0 / 2 ** lev
        cand = np.nonzero((t["level"] == lev) & (t["npts"] > 0))[0]
        b = int(rng.choice(cand))
        ctr = c0 - 0.5 * side0 + (t["coord"][b] + 0.5) * side
        inside = np.all(np.abs(x - ctr[:, None]) <= 0.5 * side, axis=0)
        dofs = np.nonzero(inside)[0]
        ng = rss.proxy_count(side, s.k, s.eps)
        pout, pin, ng2 = rss.proxy_block(x, s.normals, s.weights, s.k, s.eta, s.eps, ctr, side, dofs)
        assert ng2 == ng
        ref = np.vstack([pout, pin])
        got = fm.proxy_block(x, s.normals, s.weights, s.k, s.eta, dofs, ctr, rss.PROXY_RADIUS * side,
                             ng).cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        say("proxy rows level", lev, "shape", ref.shape, "max rel err", err)
        assert err <= 1e-13
