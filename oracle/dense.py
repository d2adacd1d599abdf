"""Dense scaled Nystrom system and its direct solution (oracle; test infrastructure).

Section 3, eqs. (disc1) and (disc3), with alpha = 1/2 and weights w_ij = w_j, or, for the
pairs listed in an optional correction table (locally corrected quadrature, target-dependent
weights w_ij = w_j (1 + a_ij), i != j):
    A~_ii = 1/2,    A~_ij = sqrt(w_i) K(x_i, x_j) w_ij / sqrt(w_j)   (i != j),
acting on the scaled unknowns sigma~_j = sqrt(w_j) sigma_j with right-hand side
b~_i = sqrt(w_i) f(x_i). The exact discrete solution is x* = A~^{-1} b~, obtained here
by LAPACK's partial-pivoting LU (scipy.linalg.lu_factor / lu_solve).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernel


def apply_corrections(blk, rows, cols, corr):
    """Multiply the entries of the block A~[rows, cols] that the correction table lists by
    (1 + a_ij). corr = (row_ptr, col, a): CSR by target row i, sources j, factors a_ij."""
    if corr is None:
        return blk
    row_ptr, ccol, ca = corr
    rows, cols = np.asarray(rows), np.asarray(cols)
    cpos = {int(j): q for q, j in enumerate(cols)}
    for p, i in enumerate(rows):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            q = cpos.get(int(ccol[e]))
            if q is not None and int(ccol[e]) != int(i):
                blk[p, q] *= 1.0 + ca[e]
    return blk


def system_matrix(x, nrm, w, k, eta, rows=None, cols=None, corr=None):
    """Block A~[rows, cols] of the scaled CFIE matrix (all of it by default), with the
    correction table's target-dependent weights when one is given."""
    n = x.shape[1]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    cols = np.arange(n) if cols is None else np.asarray(cols)
    out = np.empty((rows.size, cols.size), dtype=np.complex128)
    sw = np.sqrt(w)
    step = 2048
    for r0 in range(0, rows.size, step):
        ri = rows[r0:r0 + step]
        same = ri[:, None] == cols[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            blk = kernel.cfie(x[:, ri], x[:, cols], nrm[:, cols], k, eta)
        blk = sw[ri][:, None] * blk * sw[cols][None, :]
        blk[same] = 0.5
        out[r0:r0 + step] = blk
    return apply_corrections(out, rows, cols, corr)


def derivative_matrix(x, nrm, w, k, eta, which, corr=None):
    """dA~/dk ('k') or dA~/deta ('eta'); the diagonal 1/2 does not depend on either, and the
    correction factors (1 + a_ij) carry over to the derivative."""
    n = x.shape[1]
    sw = np.sqrt(w)
    with np.errstate(divide="ignore", invalid="ignore"):
        if which == "k":
            m = kernel.cfie_dk(x, x, nrm, k, eta)
        elif which == "eta":
            m = kernel.cfie_deta(x, x, nrm, k)
        else:
            raise ValueError(which)
    m = sw[:, None] * m * sw[None, :]
    m[np.arange(n), np.arange(n)] = 0.0
    return apply_corrections(m, np.arange(n), np.arange(n), corr)


def matvec(x, nrm, w, k, eta, v, adjoint=False):
    """A~ v (or A~^H v) without storing A~: row blocks are generated and discarded."""
    n = x.shape[1]
    v = np.asarray(v, dtype=np.complex128)
    out = np.zeros_like(v)
    step = 1024
    for r0 in range(0, n, step):
        ri = np.arange(r0, min(n, r0 + step))
        blk = system_matrix(x, nrm, w, k, eta, rows=ri)
        if adjoint:
            out += blk.conj().T @ v[ri]
        else:
            out[ri] = blk @ v
    return out


class DenseLU:
    """Partial-pivoting LU of the full dense A~ (LAPACK zgetrf)."""

    def __init__(self, a):
        self.lu = sla.lu_factor(a, check_finite=False)

    def solve(self, b):
        return sla.lu_solve(self.lu, b, check_finite=False)

    def solve_adjoint(self, b):
        # trans=2 solves A^H x = b
        return sla.lu_solve(self.lu, b, trans=2, check_finite=False)
