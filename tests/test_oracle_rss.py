"""Pins of the oracle's recursive strong skeletonization (CPU only).

Checked against what the paper fixes rather than against itself:
  * whole solve vs dense partial-pivoting LU, relative error <= 10 eps (Section 4.2's
    factored inverse is eps-accurate);
  * the factored operator A_f = V_1..V_M D W_M..W_1 reproduces A~ to O(eps);
  * adjoint solve: <A_f^{-1} b, c> = <b, A_f^{-H} c> to rounding, and vs dense A~^{-H};
  * Section 4.4's invariant: the P-blocks A_PB, A_BP hold unmodified kernel entries when
    B is compressed;
  * Section 4.3/5.1: the proxy ID is as accurate for the full far-field block
    [A_FB ; A_BF^T] as the requested tolerance (brute force against all of F);
  * special cases: a single leaf (no compression) and a tolerance near machine
    precision reduce to dense LU.
"""
import numpy as np
import pytest

import synth
from oracle import dense, rss


def _rhs(s):
    return np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)


def test_solve_matches_dense_lu(sphere3k, sphere3k_dense, sphere3k_rss):
    s = sphere3k
    _, lu = sphere3k_dense
    b = _rhs(s)
    xs = lu.solve(b)
    x = sphere3k_rss.solve(b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * s.eps


def test_structure(sphere3k_rss):
    f = sphere3k_rss
    assert f.tree.nlevels >= 3
    assert len(f.factors) > 0
    assert f.n0 < f.n
    for fa in f.factors:
        assert fa.R.size + fa.S.size == fa.m
        assert np.intersect1d(fa.R, fa.N).size == 0
        assert fa.T.shape == (fa.S.size, fa.R.size)


def test_factored_operator_reproduces_matrix(sphere3k, sphere3k_dense, sphere3k_rss):
    a, _ = sphere3k_dense
    v = np.random.default_rng(3).standard_normal(sphere3k.n) * (1 - 2j)
    av = a @ v
    assert np.linalg.norm(sphere3k_rss.apply(v) - av) / np.linalg.norm(av) <= 10 * sphere3k.eps


def test_adjoint(sphere3k, sphere3k_dense, sphere3k_rss):
    _, lu = sphere3k_dense
    rng = np.random.default_rng(4)
    b = rng.standard_normal(sphere3k.n) + 1j * rng.standard_normal(sphere3k.n)
    c = rng.standard_normal(sphere3k.n) + 1j * rng.standard_normal(sphere3k.n)
    f = sphere3k_rss
    lhs = np.vdot(c, f.solve(b))
    rhs = np.vdot(f.solve_adjoint(c), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    xa = f.solve_adjoint(c)
    xs = lu.solve_adjoint(c)
    assert np.linalg.norm(xa - xs) / np.linalg.norm(xs) <= 10 * sphere3k.eps


def test_far_field_invariant_and_proxy_accuracy(sphere3k_rss):
    f = sphere3k_rss
    assert f.invariant_checked > 50
    errs = np.array([e[1] for e in f.bf_errors])
    assert errs.size > 50
    assert errs.max() <= 3 * f.eps


def test_single_leaf_is_dense_lu():
    s = synth.unit_sphere(60)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps)
    assert len(f.factors) == 0 and f.n0 == 60
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = _rhs(s)
    xs = np.linalg.solve(a, b)
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) < 1e-13


def test_tight_tolerance_is_nearly_exact():
    s = synth.unit_sphere(800, eps=1e-13)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, 1e-13, leaf_size=16)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = _rhs(s)
    xs = np.linalg.solve(a, b)
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) < 1e-11


def test_graded_ellipsoid_small():
    s = synth.graded_ellipsoid(2500, seed=2, k=3.0, eps=1e-6)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, leaf_size=32,
                      check_invariant=True)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = _rhs(s)
    xs = np.linalg.solve(a, b)
    assert len(f.factors) > 20
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) <= 10 * s.eps


def test_phase_start_schedule():
    """The colour phase taken as one concurrent step (every box of a phase classifies the DOFs
    active when the phase began): still within 10 eps of dense LU, forward and adjoint, the
    far-field blocks of every box still untouched kernel values, and the same boxes eliminated
    in the same order as the sequential schedule."""
    s = synth.graded_ellipsoid(2000, seed=2, k=3.0, eps=1e-6)
    kw = dict(leaf_size=32, check_invariant=True)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, schedule="phase_start", **kw)
    seq = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, **kw)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    lu = dense.DenseLU(a)
    b = _rhs(s)
    xs, ys = lu.solve(b), lu.solve_adjoint(b)
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) <= 10 * s.eps
    assert np.linalg.norm(f.solve_adjoint(b) - ys) / np.linalg.norm(ys) <= 10 * s.eps
    assert f.invariant_checked > 20
    assert [(g.level, g.coord) for g in f.factors] == [(g.level, g.coord) for g in seq.factors]
    # some box of this workload has a same-colour box in its Q region eliminated earlier in
    # its phase: the two schedules then see different Q rows
    assert any(g.nq != h.nq for g, h in zip(f.factors, seq.factors))


def test_separate_skeletons():
    """Separate outgoing (column) and incoming (row) skeletons, each from its own ID at a
    common rank (the larger eps-rank, so the pivot block is square): within 10 eps of dense
    LU forward and adjoint, A_f reproduces A~ to O(eps), the far-field blocks are untouched
    kernel values at every box, both proxy IDs are as accurate as brute-force IDs of the full
    far field, and the common ranks are no larger in total than the shared ones (Section 4.1:
    one T for both blocks costs a slightly larger skeleton)."""
    s = synth.graded_ellipsoid(1500, seed=2, k=3.0, eps=1e-6)
    kw = dict(leaf_size=32, check_invariant=True)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, separate=True,
                      brute_force_check=True, **kw)
    shared = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, **kw)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    lu = dense.DenseLU(a)
    b = _rhs(s)
    xs, ys = lu.solve(b), lu.solve_adjoint(b)
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) <= 10 * s.eps
    assert np.linalg.norm(f.solve_adjoint(b) - ys) / np.linalg.norm(ys) <= 10 * s.eps
    v = np.random.default_rng(2).standard_normal(s.n) * (1 - 1j)
    assert np.linalg.norm(f.apply(v) - a @ v) / np.linalg.norm(a @ v) <= 10 * s.eps
    assert f.invariant_checked > 10
    assert max(e[1] for e in f.bf_errors) <= 3 * s.eps
    assert sum(g.S.size for g in f.factors) <= sum(g.S.size for g in shared.factors)
    # the row and column skeletons really differ somewhere
    assert any(not np.array_equal(np.sort(g.S), np.sort(g.Sr)) for g in f.factors)


def _corrected_case():
    s = synth.graded_ellipsoid(2500, seed=2, k=3.0, eps=1e-6)
    corr = synth.near_corrections(s.points, seed=1, long_frac=0.03, long_factor=14.0)
    return s, corr


def test_corrected_matrix_entries():
    """Listed pairs are the kernel entries times (1 + a_ij); every other entry and the
    diagonal are unchanged; the derivative matrices carry the same factors."""
    s = synth.unit_sphere(400)
    corr = synth.near_corrections(s.points, seed=3)
    a0 = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    a1 = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta, corr=corr)
    rp, cc, ca = corr
    fac = np.ones_like(a0)
    for i in range(s.n):
        for e in range(rp[i], rp[i + 1]):
            if cc[e] != i:
                fac[i, cc[e]] = 1.0 + ca[e]
    assert np.array_equal(a1, a0 * fac)
    assert np.all(np.diag(a1) == 0.5)
    d0 = dense.derivative_matrix(s.points, s.normals, s.weights, s.k, s.eta, "k")
    d1 = dense.derivative_matrix(s.points, s.normals, s.weights, s.k, s.eta, "k", corr=corr)
    assert np.array_equal(d1, d0 * fac)


def test_quadrature_corrections_spill_over():
    """Section 5.3: corrections that reach a box's far field move the linked owner into Q.
    With that rule the factorization stays within 10 eps of dense LU (forward and adjoint),
    no correction ever links a box to its P region, and the proxy IDs are as accurate as the
    brute-force IDs of the full far field. Without it (spill=False) the proxy surface misses
    the corrected entries: brute-force ID errors far above eps and a worse solve."""
    s, corr = _corrected_case()
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta, corr=corr)
    lu = dense.DenseLU(a)
    b = _rhs(s)
    xs, ys = lu.solve(b), lu.solve_adjoint(b)
    kw = dict(leaf_size=32, brute_force_check=True, schedule="phase_start", corr=corr)
    f = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, check_invariant=True, **kw)
    assert f.spill_count > 0
    assert np.linalg.norm(f.solve(b) - xs) / np.linalg.norm(xs) <= 10 * s.eps
    assert np.linalg.norm(f.solve_adjoint(b) - ys) / np.linalg.norm(ys) <= 10 * s.eps
    assert max(e[1] for e in f.bf_errors) <= 3 * s.eps
    off = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, spill=False, **kw)
    assert max(e[1] for e in off.bf_errors) > 30 * s.eps
    assert np.linalg.norm(off.solve(b) - xs) > np.linalg.norm(f.solve(b) - xs)


def test_empty_correction_table_is_the_plain_method():
    s = synth.unit_sphere(1500)
    empty = (np.zeros(s.n + 1, np.int64), np.zeros(0, np.int64), np.zeros(0))
    f0 = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, leaf_size=32)
    f1 = rss.RSSFactor(s.points, s.normals, s.weights, s.k, s.eta, s.eps, leaf_size=32, corr=empty)
    b = _rhs(s)
    assert np.array_equal(f0.solve(b), f1.solve(b)) and f1.spill_count == 0
