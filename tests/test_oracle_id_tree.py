"""Pins of the oracle's interpolative decomposition and octree (CPU only).

ID (Section 4.1, Definition; greedy CPQR): the truncation error of greedy CPQR is the
norm of the trailing block R22, each of whose columns is no longer than the first
rejected pivot, so ||A_R - A_S T||_2 <= sqrt(r) eps |R_00|. Pivot order is compared with
LAPACK's zgeqp3 (scipy.linalg.qr(pivoting=True)).

Octree (Section 4, opening): leaf capacity, partition of the points, geometric
containment, and the level restriction checked by brute force over all leaf pairs.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import idqr
from oracle.tree import Tree, touching


def _graded(rows, cols, decay, seed):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols)))
    v, _ = np.linalg.qr(rng.standard_normal((cols, cols)) + 1j * rng.standard_normal((cols, cols)))
    sv = decay ** np.arange(cols)
    return (u * sv) @ v.conj().T, sv


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_id_error_bound_and_rank(eps):
    a, sv = _graded(300, 60, 0.7, seed=11)
    S, Rd, T = idqr.interp_decomp(a, eps)
    piv, R, s = idqr.cpqr(a, eps)
    err = np.linalg.norm(a[:, Rd] - a[:, S] @ T, 2) if Rd.size else 0.0
    assert err <= np.sqrt(max(Rd.size, 1)) * eps * abs(R[0, 0]) * (1 + 1e-8)
    # sigma_{s+1} <= ||R22||_2 <= sqrt(r) eps |R_00| <= sqrt(r m) eps sigma_1: every singular
    # value above that level is captured; CPQR may keep a few more columns than the SVD.
    m = a.shape[1]
    must = int(np.sum(sv > np.sqrt(Rd.size * m) * eps * sv[0]))
    assert must <= S.size <= int(np.sum(sv > eps * sv[0])) + 8


def test_id_pivots_match_lapack():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((80, 25)) + 1j * rng.standard_normal((80, 25))
    a = a * np.linspace(3.0, 0.5, 25)[None, :]
    piv, R, s = idqr.cpqr(a, 1e-14)
    q2, r2, p2 = sla.qr(a, pivoting=True, mode="economic")
    assert s == 25
    assert np.array_equal(piv, p2)
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(r2)), rtol=1e-12)


def test_id_exact_low_rank():
    rng = np.random.default_rng(7)
    b = rng.standard_normal((50, 4)) + 1j * rng.standard_normal((50, 4))
    c = rng.standard_normal((4, 30)) + 1j * rng.standard_normal((4, 30))
    a = b @ c
    S, Rd, T = idqr.interp_decomp(a, 1e-10)
    assert S.size == 4
    assert np.linalg.norm(a[:, Rd] - a[:, S] @ T) < 1e-12 * np.linalg.norm(a)


def test_id_zero_matrix_and_full_rank():
    S, Rd, T = idqr.interp_decomp(np.zeros((5, 3), complex), 1e-6)
    assert S.size == 0 and Rd.size == 3
    a = np.eye(4, dtype=complex)
    S, Rd, T = idqr.interp_decomp(a, 1e-6)
    assert S.size == 4 and Rd.size == 0
    assert list(S) == [0, 1, 2, 3]  # equal norms: lowest index first


def _check_tree(t, x, s):
    n = x.shape[1]
    leaves = t.leaves()
    seen = np.zeros(n, dtype=int)
    for b in leaves:
        seen[t.pts[b]] += 1
        assert t.pts[b].size <= s
    assert np.all(seen == 1)
    # containment: every point lies in the closed box of its leaf
    for b in leaves:
        if t.pts[b].size == 0:
            continue
        lo = t.root_lo + t.coord[b] * t.box_side(b)
        hi = lo + t.box_side(b)
        p = x[:, t.pts[b]]
        tol = 1e-12 * t.side
        assert np.all(p >= lo[:, None] - tol) and np.all(p <= hi[:, None] + tol)
    # non-leaves: split because they were over capacity or to restore the level restriction
    for b in range(len(t.level)):
        if not t.is_leaf[b]:
            kids = t.children[b]
            assert sum(t.pts[c].size for c in kids) == t.pts[b].size
    # level restriction, brute force over all leaf pairs
    L = [(int(t.level[b]), tuple(t.coord[b])) for b in leaves]
    for i in range(len(L)):
        for j in range(i + 1, len(L)):
            if abs(L[i][0] - L[j][0]) > 1 and touching(L[i][0], L[i][1], L[j][0], L[j][1]):
                raise AssertionError(f"level restriction violated: {L[i]} {L[j]}")
    # tree order: each box's points are contiguous
    for b in range(len(t.level)):
        r = np.sort(t.rank[t.pts[b]])
        if r.size:
            assert r[-1] - r[0] + 1 == r.size


def test_tree_sphere():
    s = synth.unit_sphere(3000)
    t = Tree(s.points, 64)
    _check_tree(t, s.points, 64)


def test_tree_graded_needs_balancing():
    s = synth.graded_ellipsoid(4000, seed=2)
    t = Tree(s.points, 16)
    _check_tree(t, s.points, 16)
    assert t.nlevels >= 6


def test_tree_single_leaf():
    s = synth.unit_sphere(50)
    t = Tree(s.points, 64)
    assert len(t.level) == 1 and t.nlevels == 1
