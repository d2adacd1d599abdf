"""Interpolative decomposition by greedy column-pivoted QR (oracle; test infrastructure).

Section 4.1, Definition (interpolative decomposition): split the columns J of A into
skeleton columns S and redundant columns R with an interpolation matrix T such that
||A_R - A_S T|| <= eps ||A||. The paper computes it with the standard greedy
column-pivoted QR: at each step the remaining column of largest 2-norm is moved
to the front and eliminated with a Householder reflector.

Readings (the paper fixes only the relative spectral-norm accuracy):
  * Truncation: the rank s is the number of pivots k with |R_kk| > eps |R_00|
    (|R_00| is the largest column norm); greedy pivots are non-increasing, so the
    process stops at the first pivot that fails.
  * Ties in the column norm go to the lowest original column index.
  * T = R11^{-1} R12 by back-substitution, R11 = R[:s, :s], R12 = R[:s, s:].

Column norms are recomputed exactly from the trailing rows at every step (no
downdating). `cpqr(..., margins=True)` also reports how close each decision came to going
the other way (used to recognise near-ties when comparing with other implementations):
  gap2  = min over the pivot steps of (n1^2 - n2^2) / nmax^2, n1 >= n2 the two largest
          remaining column norms at that step and nmax the largest initial column norm;
  gap1  = the same minimum of (n1 - n2) / nmax;
  trunc2, trunc1 = |n^2 - (eps R_00)^2| / nmax^2 and |n - eps R_00| / nmax, minimised over
          the last accepted and the first rejected pivot (the truncation decision).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cpqr(a, eps, max_rank=None, margins=False):
    """Greedy CPQR of a (rows x m), stopped at the relative tolerance eps.

    Returns (piv, R, s): piv is the column order (first s are skeletons), R the
    (min(rows, m) x m) upper-trapezoidal factor in pivoted column order, s the rank;
    with margins=True a fourth item, the dict of decision margins described above.
    """
    a = np.array(a, dtype=np.complex128, copy=True)
    rows, m = a.shape
    piv = np.arange(m)
    kmax = min(rows, m) if max_rank is None else min(rows, m, max_rank)
    r00 = None
    s = 0
    nmax = float(np.linalg.norm(a, axis=0).max()) if a.size else 0.0
    mg = {"gap2": np.inf, "gap1": np.inf, "trunc2": np.inf, "trunc1": np.inf}

    def note_trunc(nk):
        if nmax > 0 and r00 is not None:
            t = eps * r00
            mg["trunc2"] = min(mg["trunc2"], abs(nk * nk - t * t) / nmax ** 2)
            mg["trunc1"] = min(mg["trunc1"], abs(nk - t) / nmax)

    for k in range(kmax):
        norms = np.linalg.norm(a[k:, k:], axis=0)
        # largest norm; ties -> lowest original index among the remaining columns
        best = norms.max()
        cand = np.nonzero(norms == best)[0]
        j = k + cand[np.argmin(piv[k + cand])]
        if j != k:
            a[:, [k, j]] = a[:, [j, k]]
            piv[[k, j]] = piv[[j, k]]
        nk = norms[j - k]
        if k == 0:
            r00 = nk
            if r00 == 0.0:
                s = 0
                break
        else:
            note_trunc(nk)
            if nk <= eps * r00:
                s = k
                break
        if norms.size > 1 and nmax > 0:
            n1, n2 = np.sort(norms)[-2:][::-1]
            mg["gap2"] = min(mg["gap2"], (n1 * n1 - n2 * n2) / nmax ** 2)
            mg["gap1"] = min(mg["gap1"], (n1 - n2) / nmax)
        # Householder reflector mapping a[k:, k] to -e^{i arg a_kk} ||.|| e_1
        v = a[k:, k].copy()
        alpha = v[0]
        phase = alpha / abs(alpha) if alpha != 0 else 1.0
        v[0] += phase * nk
        vn = np.linalg.norm(v)
        if vn > 0:
            v /= vn
            a[k:, k:] -= 2.0 * np.outer(v, v.conj() @ a[k:, k:])
        a[k + 1:, k] = 0.0
        s = k + 1
    R = np.triu(a[:min(rows, m), :])
    if margins:
        return piv, R, s, mg
    return piv, R, s


def interp_decomp(a, eps, margins=False):
    """eps-accurate ID of the columns of a: returns (S, Rd, T) as column positions,
    with a[:, Rd] ~= a[:, S] @ T (T is s x r); with margins=True also cpqr's margins."""
    piv, R, s, mg = cpqr(a, eps, margins=True)
    m = a.shape[1]
    S, Rd = piv[:s].copy(), piv[s:].copy()
    if s == 0:
        T = np.zeros((0, m), dtype=np.complex128)
    else:
        T = sla.solve_triangular(R[:s, :s], R[:s, s:m], lower=False)
    return (S, Rd, T, mg) if margins else (S, Rd, T)
