"""Helmholtz Green's function and combined-field kernel (oracle; test infrastructure).

Section 3, eq. (greenfunhelm): G(x, y) = e^{ik|x-y|} / (4 pi |x-y|).
Section 3, eq. (comb_ref): K(x, y) = n(y) . grad_y G(x, y) - i k G(x, y); the coupling
constant k in front of the single layer is generalised to eta (K = D - i eta S).

Written out with rho = |x - y| and d = x - y:
    grad_y G = e^{ik rho} (1 - ik rho) d / (4 pi rho^3)
so  K(x, y) = e^{ik rho} / (4 pi rho^3) * [ (1 - ik rho) (d . n(y)) - i eta rho^2 ].

Derivatives used by the gradient of the far-field loss:
    dG/dk = i rho G
    d/dk [n(y) . grad_y G] = k e^{ik rho} (d . n(y)) / (4 pi rho)
    dK/deta = -i G
"""
from __future__ import annotations

import math

import numpy as np


def _diff(x, y):
    """x (3, m), y (3, n) -> d (3, m, n) with d[:, i, j] = x_i - y_j, rho (m, n)."""
    d = x[:, :, None] - y[:, None, :]
    rho = np.sqrt(np.sum(d * d, axis=0))
    return d, rho


def green(x, y, k):
    """G(x_i, y_j) for targets x (3, m) and sources y (3, n); eq. (greenfunhelm)."""
    _, rho = _diff(x, y)
    return np.exp(1j * k * rho) / (4.0 * math.pi * rho)


def double_layer(x, y, ny, k):
    """n(y_j) . grad_y G(x_i, y_j); the double-layer part of eq. (comb_ref)."""
    d, rho = _diff(x, y)
    dn = np.einsum("aij,aj->ij", d, ny)
    return np.exp(1j * k * rho) * (1.0 - 1j * k * rho) * dn / (4.0 * math.pi * rho ** 3)


def cfie(x, y, ny, k, eta):
    """Combined-field kernel K(x_i, y_j) = D - i eta S; eq. (comb_ref) with ik -> i eta."""
    return double_layer(x, y, ny, k) - 1j * eta * green(x, y, k)


def cfie_dk(x, y, ny, k, eta):
    """dK/dk at fixed eta: k e^{ik rho}(d.n)/(4 pi rho) - i eta * i rho G."""
    d, rho = _diff(x, y)
    dn = np.einsum("aij,aj->ij", d, ny)
    e = np.exp(1j * k * rho)
    ddl = k * e * dn / (4.0 * math.pi * rho)
    dg = 1j * rho * e / (4.0 * math.pi * rho)
    return ddl - 1j * eta * dg


def cfie_deta(x, y, ny, k):
    """dK/deta = -i G."""
    return -1j * green(x, y, k)
