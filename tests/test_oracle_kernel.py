"""Pins of the oracle's kernel and dense system against closed forms (CPU only).

Section 3, eqs. (greenfunhelm), (comb_ref), (disc3). None of these tests re-types the
oracle's formula: each compares it with an independent derivation (finite differences,
the Laplace limit, a one-dimensional reduction of the sphere integrals, spherical
Bessel functions from scipy, or Green's representation formula).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import synth
from oracle import dense, kernel


def _rand_pairs(seed, m=20):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((3, m))
    y = rng.standard_normal((3, m)) + 2.5
    n = rng.standard_normal((3, m))
    n /= np.linalg.norm(n, axis=0)
    return x, y, n


def test_green_symmetric():
    x, y, _ = _rand_pairs(0)
    g1 = kernel.green(x, y, 1.7)
    g2 = kernel.green(y, x, 1.7)
    assert np.allclose(g1, g2.T, rtol=1e-15, atol=0)


def test_double_layer_matches_finite_difference_of_green():
    # n(y) . grad_y G by central differences of G in y (step h, error O(h^2)).
    x, y, n = _rand_pairs(1)
    k, h = 2.3, 1e-5
    dl = kernel.double_layer(x, y, n, k)
    for j in range(y.shape[1]):
        xi = x
        yp = y[:, j:j + 1] + h * n[:, j:j + 1]
        ym = y[:, j:j + 1] - h * n[:, j:j + 1]
        fd = (kernel.green(xi, yp, k) - kernel.green(xi, ym, k))[:, 0] / (2 * h)
        assert np.allclose(dl[:, j], fd, rtol=1e-8, atol=1e-12)


def test_laplace_limit():
    # k = 0: G = 1/(4 pi r), n(y).grad_y G = (x-y).n / (4 pi r^3) (textbook Laplace kernels).
    x, y, n = _rand_pairs(2)
    d = x[:, :, None] - y[:, None, :]
    r = np.sqrt(np.sum(d * d, axis=0))
    assert np.allclose(kernel.green(x, y, 0.0), 1 / (4 * math.pi * r), rtol=1e-15)
    dn = np.einsum("aij,aj->ij", d, n)
    assert np.allclose(kernel.double_layer(x, y, n, 0.0), dn / (4 * math.pi * r ** 3), rtol=1e-14)


def test_k_derivative_matches_finite_difference():
    x, y, n = _rand_pairs(3)
    k, eta, h = 1.3, 0.7, 1e-6
    fd = (kernel.cfie(x, y, n, k + h, eta) - kernel.cfie(x, y, n, k - h, eta)) / (2 * h)
    assert np.allclose(kernel.cfie_dk(x, y, n, k, eta), fd, rtol=1e-7, atol=1e-12)
    fd_eta = (kernel.cfie(x, y, n, k, eta + h) - kernel.cfie(x, y, n, k, eta - h)) / (2 * h)
    assert np.allclose(kernel.cfie_deta(x, y, n, k), fd_eta, rtol=1e-7, atol=1e-12)


def _sphere_point_at_chord(rho):
    # point on the unit sphere at chord distance rho from the north pole (0,0,1)
    c = 1.0 - rho * rho / 2.0
    s = math.sqrt(max(0.0, 1.0 - c * c))
    return np.array([[s], [0.0], [c]])


@pytest.mark.parametrize("k", [0.5, 1.0, 3.0])
def test_unit_sphere_constant_density_integrals(k):
    """On the unit sphere the area of {y : |x-y| in [rho, rho+d rho]} is 2 pi rho d rho, so
    S[1] = int_0^2 G 2 pi rho d rho = (e^{2ik} - 1)/(2ik) and
    D[1] = int_0^2 n(y).grad_y G 2 pi rho d rho = e^{2ik}/2 - (e^{2ik} - 1)/(2ik)
    (derived by hand from the kernel's definition; the integrals are evaluated through the
    oracle's kernel functions at actual sphere points)."""
    x0 = np.array([[0.0], [0.0], [1.0]])

    def integrand(rho, which, part):
        y = _sphere_point_at_chord(rho)
        if which == "S":
            v = kernel.green(x0, y, k)[0, 0]
        else:
            v = kernel.double_layer(x0, y, y, k)[0, 0]
        v = v * 2 * math.pi * rho
        return v.real if part == 0 else v.imag

    s_num = complex(si.quad(integrand, 0, 2, args=("S", 0), epsabs=1e-13, limit=200)[0],
                    si.quad(integrand, 0, 2, args=("S", 1), epsabs=1e-13, limit=200)[0])
    d_num = complex(si.quad(integrand, 0, 2, args=("D", 0), epsabs=1e-13, limit=200)[0],
                    si.quad(integrand, 0, 2, args=("D", 1), epsabs=1e-13, limit=200)[0])
    e2 = np.exp(2j * k)
    s_cf = (e2 - 1) / (2j * k)
    d_cf = e2 / 2 - (e2 - 1) / (2j * k)
    assert abs(s_num - s_cf) < 1e-10
    assert abs(d_num - d_cf) < 1e-10


def _sph_h(l, k, derivative=False):
    return sp.spherical_jn(l, k, derivative) + 1j * sp.spherical_yn(l, k, derivative)


def _cfie_eigenvalue(l, k, eta):
    """lambda_l = 1/2 + (ik^2/2)(j_l h_l' + j_l' h_l) + eta k j_l h_l on the unit sphere
    (addition theorem for G; the principal value is the mean of the two one-sided limits)."""
    j, jd = sp.spherical_jn(l, k), sp.spherical_jn(l, k, True)
    h, hd = _sph_h(l, k), _sph_h(l, k, True)
    return 0.5 + 0.5j * k * k * (j * hd + jd * h) + eta * k * j * h


def test_sphere_eigenvalue_l0_two_derivations_agree():
    for k, eta in [(1.0, 1.0), (2.0, 0.5), (5.0, 5.0)]:
        e2 = np.exp(2j * k)
        s1 = (e2 - 1) / (2j * k)
        d1 = e2 / 2 - s1
        assert abs(_cfie_eigenvalue(0, k, eta) - (0.5 + d1 - 1j * eta * s1)) < 1e-12


def test_sphere_eigenvalue_printed_values():
    # k = eta = 1: lambda_0 = 0.54535 - 0.70807i (five digits).
    lam0 = _cfie_eigenvalue(0, 1.0, 1.0)
    assert abs(lam0 - (0.54535 - 0.70807j)) < 1e-5


@pytest.mark.parametrize("l", [0, 1, 2])
def test_sphere_spectrum_discrete(l):
    """A~ (sqrt(w) Y_l0) ~ lambda_l sqrt(w) Y_l0 on the Fibonacci sphere. The punctured
    Nystrom rule is only O(h) accurate, so the error must be small and shrink with n."""
    errs = []
    for n in (750, 3000):
        s = synth.unit_sphere(n)
        a = dense.system_matrix(s.points, s.normals, s.weights, 1.0, 1.0)
        z = s.points[2]
        y = sp.eval_legendre(l, z)
        v = np.sqrt(s.weights) * y
        lam = _cfie_eigenvalue(l, 1.0, 1.0)
        errs.append(np.linalg.norm(a @ v - lam * v) / np.linalg.norm(v))
    assert errs[1] < 0.05
    assert errs[1] < 0.75 * errs[0]


def test_green_representation_exterior_field(sphere3k, sphere3k_dense):
    """Section 6.1's check: Dirichlet data from an interior point source; the exterior
    combined-field potential of the solved density must reproduce the source's field."""
    src = (0.1, 0.2, 0.3)
    t = synth.exterior_targets(50, seed=0)
    ref = kernel.green(t, np.array(src)[:, None], sphere3k.k)[:, 0]

    def field_error(s, lu):
        b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k, src)
        sig = lu.solve(b)
        u = kernel.cfie(t, s.points, s.normals, s.k, s.eta) @ (np.sqrt(s.weights) * sig)
        return np.linalg.norm(u - ref) / np.linalg.norm(ref), sig

    s = sphere3k
    rel, sig = field_error(s, sphere3k_dense[1])
    small = synth.unit_sphere(750)
    rel_small, _ = field_error(small, dense.DenseLU(dense.system_matrix(
        small.points, small.normals, small.weights, small.k, small.eta)))
    # first-order convergence of the punctured rule: ~2x smaller error for 4x more points
    assert rel < 5e-2
    assert rel < 0.7 * rel_small
    # a sign error in either kernel term gives an O(1) mismatch
    bad = kernel.cfie(t, s.points, -s.normals, s.k, s.eta) @ (np.sqrt(s.weights) * sig)
    assert np.linalg.norm(bad - ref) / np.linalg.norm(ref) > 0.2


def test_dense_matrix_diagonal_and_symmetry(sphere3k):
    s = synth.unit_sphere(400)
    a = dense.system_matrix(s.points, s.normals, s.weights, 1.0, 1.0)
    assert np.all(a[np.arange(400), np.arange(400)] == 0.5)
    # single-layer part is symmetric; with eta only (no double layer at k=0 on a sphere
    # the double layer is not symmetric) check the eta-derivative block instead
    d = dense.derivative_matrix(s.points, s.normals, s.weights, 1.0, 1.0, "eta")
    assert np.allclose(d, d.T, rtol=1e-14, atol=0)


def test_matvec_matches_dense():
    s = synth.unit_sphere(700)
    a = dense.system_matrix(s.points, s.normals, s.weights, 1.0, 1.0)
    v = np.random.default_rng(0).standard_normal(700) * (1 + 1j)
    assert np.allclose(dense.matvec(s.points, s.normals, s.weights, 1.0, 1.0, v), a @ v, rtol=1e-13)
    assert np.allclose(dense.matvec(s.points, s.normals, s.weights, 1.0, 1.0, v, adjoint=True),
                       a.conj().T @ v, rtol=1e-13)
