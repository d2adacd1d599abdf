"""Differentiable solve and far-field pattern (adjoint gradients through the factors).

With sigma~ = A~^{-1} b~ and an upstream gradient g in PyTorch's complex convention
(g = dL/dRe x + i dL/dIm x), the reverse pass needs one adjoint solve:
    lambda = A~^{-H} g,   grad_b = lambda,
    dL/dk  = -Re(lambda^H (dA~/dk) sigma~),   dL/deta = -Re(lambda^H (dA~/deta) sigma~),
where the derivative products are the exact on-the-fly matvecs. For the far-field pattern
F = C sigma~ (Section 6.3's pattern of the combined-field potential):
    grad_sigma = C^H g_F,   dL/dk = Re(g_F^H (dC/dk) sigma~),   dL/deta = Re(g_F^H (dC/deta) sigma~).
The factorization is built at fixed (k, eta); the tensors k and eta passed here only
carry gradients and must hold the same values.
"""
from __future__ import annotations

import torch

__all__ = ["FMMLUSolve", "FarField", "solve", "far_field", "plane_wave_rhs", "far_field_loss"]


def _check_params(factor, k, eta):
    if abs(float(k) - factor.k) > 1e-14 * max(1.0, abs(factor.k)) or \
            abs(float(eta) - factor.eta) > 1e-14 * max(1.0, abs(factor.eta)):
        raise ValueError(f"k, eta = ({float(k)}, {float(eta)}) differ from the factorization's "
                         f"({factor.k}, {factor.eta})")


def _shape_of(v):
    return v.shape if isinstance(v, torch.Tensor) else None


def _as_param_grad(g, shape):
    return g if shape is None else g.reshape(shape)


def _solve(factor, b, adjoint, refine_tol):
    if refine_tol is None:
        return factor.solve_adjoint(b) if adjoint else factor.solve(b)
    x, _, _ = factor.solve_refined(b, adjoint=adjoint, tol=refine_tol)
    return x


class FMMLUSolve(torch.autograd.Function):
    """x = A~^{-1} b with gradients for b, k and eta (refine_tol: use refined solves)."""

    @staticmethod
    def forward(ctx, b, k, eta, factor, refine_tol=None):
        _check_params(factor, k, eta)
        x = _solve(factor, b.detach().contiguous(), False, refine_tol)
        ctx.save_for_backward(x)
        ctx.factor, ctx.refine_tol = factor, refine_tol
        ctx.kshape, ctx.eshape = _shape_of(k), _shape_of(eta)
        return x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        f = ctx.factor
        lam = _solve(f, g.contiguous(), True, ctx.refine_tol)
        gk = geta = None
        if ctx.needs_input_grad[1]:
            gk = _as_param_grad(-torch.real(torch.vdot(lam, f.matvec(x, 2))), ctx.kshape)
        if ctx.needs_input_grad[2]:
            geta = _as_param_grad(-torch.real(torch.vdot(lam, f.matvec(x, 3))), ctx.eshape)
        return lam, gk, geta, None, None


class FarField(torch.autograd.Function):
    """F = C sigma~ over unit directions dirs (3, ndir), with gradients for sigma~, k, eta."""

    @staticmethod
    def forward(ctx, sigma, k, eta, factor, dirs):
        _check_params(factor, k, eta)
        sigma = sigma.detach().contiguous()
        F = factor.farfield(dirs, sigma, 0)
        ctx.save_for_backward(sigma)
        ctx.factor, ctx.dirs = factor, dirs
        ctx.kshape, ctx.eshape = _shape_of(k), _shape_of(eta)
        return F

    @staticmethod
    def backward(ctx, gF):
        (sigma,) = ctx.saved_tensors
        f, dirs = ctx.factor, ctx.dirs
        gF = gF.contiguous()
        gs = f.farfield(dirs, gF, 1) if ctx.needs_input_grad[0] else None
        gk = geta = None
        if ctx.needs_input_grad[1]:
            gk = _as_param_grad(torch.real(torch.vdot(gF, f.farfield(dirs, sigma, 2))), ctx.kshape)
        if ctx.needs_input_grad[2]:
            geta = _as_param_grad(torch.real(torch.vdot(gF, f.farfield(dirs, sigma, 3))), ctx.eshape)
        return gs, gk, geta, None, None


def solve(factor, b, k, eta, refine_tol=None):
    return FMMLUSolve.apply(b, k, eta, factor, refine_tol)


def far_field(factor, sigma, k, eta, dirs):
    return FarField.apply(sigma, k, eta, factor, dirs)


def plane_wave_rhs(points, weights, k, d):
    """b~ = -sqrt(w) e^{ik d.x} as torch ops (its k-dependence is differentiated by torch).

    points: (3, n) float64 CUDA tensor; weights: (n,); k: 0-dim float64 tensor; d: (3,)."""
    t = torch.as_tensor(d, dtype=torch.float64, device=points.device) @ points
    ph = torch.polar(torch.ones_like(t), k * t)
    return -torch.sqrt(weights).to(ph.dtype) * ph


def far_field_loss(factor, b, k, eta, dirs, refine_tol=None):
    """L = sum_m |F(d_m)|^2 with sigma~ = A~^{-1} b; returns (L, F)."""
    sigma = solve(factor, b, k, eta, refine_tol)
    F = far_field(factor, sigma, k, eta, dirs)
    return torch.sum(torch.abs(F) ** 2), F
