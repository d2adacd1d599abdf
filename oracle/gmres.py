"""Unpreconditioned GMRES in float64 (oracle; test infrastructure).

Where dense LU of the full matrix is out of reach (tens of thousands of unknowns), the
reference solution x* = A~^{-1} b~ of Section 3's discrete system is obtained by GMRES
(Saad and Schultz, 1986) with the exact matvec: Arnoldi with modified Gram-Schmidt and
one re-orthogonalisation pass, the small least-squares problem solved by Givens
rotations, restarts after `restart` steps. The iteration stops when the TRUE residual
||b - A x|| / ||b||, recomputed with the matvec at each restart, is <= tol. The second-kind
combined-field system is well conditioned, so the error of x is within a small multiple of
that residual.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, tol=1e-13, restart=200, maxit=2000, x0=None, log=None):
    """Solve A x = b; returns (x, relres, total_iterations). `matvec(v)` returns A v."""
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    if nb == 0.0:
        return np.zeros_like(b), 0.0, 0
    its = 0
    r = b - matvec(x) if x0 is not None else b.copy()
    rel = np.linalg.norm(r) / nb
    while rel > tol and its < maxit:
        beta = np.linalg.norm(r)
        m = min(restart, maxit - its)
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(V[j])
            for _ in range(2):  # modified Gram-Schmidt, then once more
                for i in range(j + 1):
                    h = np.vdot(V[i], w)
                    H[i, j] += h
                    w = w - h * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            # previous rotations applied to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            # rotation that zeroes H[j+1, j]
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = abs(a) / den
                ph = a / abs(a) if a != 0 else 1.0
                sn[j] = ph * np.conj(c) / den
            H[j, j] = cs[j] * a + sn[j] * c
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            est = abs(g[j + 1]) / nb
            if log is not None:
                log(its, est)
            if est <= 0.5 * tol:
                break
        # x += V_k y with H_k y = g_k (upper triangular after the rotations)
        k = j_done
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + V[:k].T @ y
        r = b - matvec(x)
        rel = np.linalg.norm(r) / nb
    return x, float(rel), its
