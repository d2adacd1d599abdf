"""Pin of the oracle's far-field operator (Section 6.3's pattern, CPU only).

The far-field pattern is defined by u(x) = e^{ikr}/r F(x^) + O(1/r^2). It is checked
against R e^{-ikR} u(R x^) evaluated with the oracle's kernel at growing R: the mismatch
must fall like 1/R. A sign error in the exponent or in either term gives an O(1) mismatch."""
import numpy as np

import synth
from oracle import farfield, kernel


def test_far_field_pattern_is_the_large_r_limit():
    s = synth.unit_sphere(300, k=2.0, eta=1.5)
    rng = np.random.default_rng(9)
    sig = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    dirs = synth.fibonacci_sphere_dirs(12)
    C = farfield.operator(dirs, s.points, s.normals, s.weights, s.k, s.eta)
    F = C @ sig
    errs = []
    for R in (1e3, 1e4):
        t = R * dirs
        u = kernel.cfie(t, s.points, s.normals, s.k, s.eta) @ (np.sqrt(s.weights) * sig)
        approx = R * np.exp(-1j * s.k * R) * u
        errs.append(np.linalg.norm(approx - F) / np.linalg.norm(F))
    assert errs[1] < 2e-3
    assert errs[1] < 0.2 * errs[0]


def test_far_field_derivatives_match_finite_differences():
    s = synth.unit_sphere(200)
    dirs = synth.fibonacci_sphere_dirs(5)
    k, eta, h = 1.7, 0.9, 1e-6
    dk = (farfield.operator(dirs, s.points, s.normals, s.weights, k + h, eta)
          - farfield.operator(dirs, s.points, s.normals, s.weights, k - h, eta)) / (2 * h)
    assert np.allclose(farfield.operator_dk(dirs, s.points, s.normals, s.weights, k, eta), dk,
                       rtol=1e-7, atol=1e-12)
    de = (farfield.operator(dirs, s.points, s.normals, s.weights, k, eta + h)
          - farfield.operator(dirs, s.points, s.normals, s.weights, k, eta - h)) / (2 * h)
    assert np.allclose(farfield.operator_deta(dirs, s.points, s.normals, s.weights, k), de,
                       rtol=1e-7, atol=1e-12)


def _grad_case():
    s = synth.unit_sphere(500, k=3.0, eta=2.0)
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    return s, d, synth.fibonacci_sphere_dirs(16)


def test_dense_gradient_wrt_rhs_is_exact_for_the_quadratic_loss():
    """L is a quadratic form in b~, so the central difference along any complex direction
    equals Re(grad_b^H delta) up to rounding, for every step size."""
    s, d, dirs = _grad_case()
    g = farfield.dense_loss_gradients(s.points, s.normals, s.weights, s.k, s.eta, d, dirs)
    rng = np.random.default_rng(5)
    delta = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    for t in (1e-2, 1.0):
        lp = farfield.dense_loss(s.points, s.normals, s.weights, s.k, s.eta, d, dirs, b=g["b"] + t * delta)
        lm = farfield.dense_loss(s.points, s.normals, s.weights, s.k, s.eta, d, dirs, b=g["b"] - t * delta)
        fd = (lp - lm) / (2 * t)
        assert abs(fd - np.real(np.vdot(g["grad_b"], delta))) <= 1e-10 * abs(fd)


def test_dense_gradient_wrt_k_and_eta_matches_finite_differences():
    """dL/dk collects the rhs, the matrix and the far-field operator terms; dropping or
    mis-signing any of them is far above the O(h^2) difference error."""
    s, d, dirs = _grad_case()
    g = farfield.dense_loss_gradients(s.points, s.normals, s.weights, s.k, s.eta, d, dirs)
    h = 1e-4 * s.k
    lp = farfield.dense_loss(s.points, s.normals, s.weights, s.k + h, s.eta, d, dirs)
    lm = farfield.dense_loss(s.points, s.normals, s.weights, s.k - h, s.eta, d, dirs)
    fd_k = (lp - lm) / (2 * h)
    assert abs(fd_k - g["dL_dk"]) <= 1e-6 * abs(fd_k)
    h = 1e-4 * s.eta
    lp = farfield.dense_loss(s.points, s.normals, s.weights, s.k, s.eta + h, d, dirs)
    lm = farfield.dense_loss(s.points, s.normals, s.weights, s.k, s.eta - h, d, dirs)
    fd_e = (lp - lm) / (2 * h)
    assert abs(fd_e - g["dL_deta"]) <= 1e-6 * abs(fd_e)
    # each of the three k terms matters at this size
    assert abs(g["dL_dk"]) > 1e-3 * g["L"]
