"""Far-field pattern of the combined-field potential and a far-field loss (oracle).

Section 6.3 defines the far-field pattern F[u] by u(x) = e^{ikr}/r F[u](x^) + O(1/r^2)
and computes the monostatic cross section from it. From the large-|x| form of the
kernel, grad_y G -> -ik x^ G and G -> e^{ik|x|}/(4 pi |x|) e^{-ik x^.y}, so the
pattern of u = sum_j K(x, x_j) sqrt(w_j) sigma~_j is
    F(x^) = (-i / 4 pi) sum_j sqrt(w_j) (k x^.n_j + eta) e^{-ik x^.x_j} sigma~_j.
(The paper prints the monostatic formula with exponent e^{-ik x.d}; with x^ = -d the
expression above gives (1 - n.d) e^{+ik d.x}, which is taken as the intended sign.)

Loss L = sum_m |F(x^_m)|^2. With sigma~ = A~^{-1} b~ and PyTorch's convention for
complex gradients (g = dL/dRe + i dL/dIm):
    lambda   = A~^{-H} C^H (2F)                     (gradient with respect to b~)
    dL/dk    = Re(lambda^H (db~/dk - dA~/dk sigma~)) + 2 Re(F^H dC/dk sigma~)
    dL/deta  = Re(lambda^H (-dA~/deta sigma~)) + 2 Re(F^H dC/deta sigma~)
"""
from __future__ import annotations

import math

import numpy as np


def operator(dirs, x, nrm, w, k, eta):
    """C (m x n): F = C sigma~ for unit directions dirs (3, m)."""
    ph = np.exp(-1j * k * (dirs.T @ x))
    return (-1j / (4.0 * math.pi)) * np.sqrt(w)[None, :] * (k * (dirs.T @ nrm) + eta) * ph


def operator_dk(dirs, x, nrm, w, k, eta):
    dx = dirs.T @ x
    dn = dirs.T @ nrm
    ph = np.exp(-1j * k * dx)
    return (-1j / (4.0 * math.pi)) * np.sqrt(w)[None, :] * (dn - 1j * dx * (k * dn + eta)) * ph


def operator_deta(dirs, x, nrm, w, k):
    ph = np.exp(-1j * k * (dirs.T @ x))
    return (-1j / (4.0 * math.pi)) * np.sqrt(w)[None, :] * ph


def loss(C, sigma):
    F = C @ sigma
    return float(np.sum(np.abs(F) ** 2)), F


def plane_wave_rhs(x, w, k, d):
    """b~ = -sqrt(w) e^{ik d.x} (the scaled Dirichlet data cancelling the incident plane wave
    along unit d, Section 6.3's scattering setting) and its k-derivative."""
    d = np.asarray(d, dtype=np.float64)
    t = d @ x
    b = -np.sqrt(w) * np.exp(1j * k * t)
    return b, 1j * t * b


def dense_loss_gradients(x, nrm, w, k, eta, d, dirs):
    """Far-field loss of the plane-wave problem and its adjoint gradients, everything dense.

    sigma~ = A~^{-1} b~; F = C sigma~; L = |F|^2. Returns a dict with L, F, sigma,
    grad_b (= lambda = A~^{-H} C^H 2F), dL/dk and dL/deta (formulas in the module header),
    using the dense LU of A~ and the dense derivative matrices."""
    from . import dense

    a = dense.system_matrix(x, nrm, w, k, eta)
    lu = dense.DenseLU(a)
    b, db_dk = plane_wave_rhs(x, w, k, d)
    sigma = lu.solve(b)
    C = operator(dirs, x, nrm, w, k, eta)
    L, F = loss(C, sigma)
    lam = lu.solve_adjoint(C.conj().T @ (2.0 * F))
    dA_dk = dense.derivative_matrix(x, nrm, w, k, eta, "k")
    dA_deta = dense.derivative_matrix(x, nrm, w, k, eta, "eta")
    dC_dk = operator_dk(dirs, x, nrm, w, k, eta)
    dC_deta = operator_deta(dirs, x, nrm, w, k)
    dL_dk = np.real(np.vdot(lam, db_dk - dA_dk @ sigma)) + 2.0 * np.real(np.vdot(F, dC_dk @ sigma))
    dL_deta = np.real(np.vdot(lam, -(dA_deta @ sigma))) + 2.0 * np.real(np.vdot(F, dC_deta @ sigma))
    return {"L": L, "F": F, "sigma": sigma, "b": b, "grad_b": lam, "dL_dk": float(dL_dk),
            "dL_deta": float(dL_deta)}


def dense_loss(x, nrm, w, k, eta, d, dirs, b=None):
    """L alone (dense solve), for finite differences. b overrides the plane-wave b~."""
    from . import dense

    a = dense.system_matrix(x, nrm, w, k, eta)
    if b is None:
        b = plane_wave_rhs(x, w, k, d)[0]
    sigma = dense.DenseLU(a).solve(b)
    return loss(operator(dirs, x, nrm, w, k, eta), sigma)[0]
