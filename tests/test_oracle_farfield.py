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
