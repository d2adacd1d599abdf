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
