"""Pins of the oracle's compiled exact matvec and its float64 GMRES (CPU only).

* The compiled matvec (oracle/matvec.c) reproduces the sphere spectrum of the combined-field
  operator: A~ (sqrt(w) Y_l0) ~ lambda_l sqrt(w) Y_l0 with lambda_l from spherical Bessel
  functions (addition theorem), to the punctured rule's O(h) error, shrinking with n; its
  adjoint is the conjugate transpose (<A~ u, v> = <u, A~^H v>); it agrees with the NumPy
  dense matrix (itself pinned by closed forms) to rounding; row subsets equal full rows.
* GMRES: the solution of a well-conditioned system equals the partial-pivoting LU solution
  (LAPACK) to the requested residual times the condition number, with and without
  restarts; a zero right-hand side gives zero; the returned residual is the true one.
"""
import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import cmatvec, dense, gmres


def _cfie_eigenvalue(l, k, eta):
    j, jd = sp.spherical_jn(l, k), sp.spherical_jn(l, k, True)
    h = sp.spherical_jn(l, k) + 1j * sp.spherical_yn(l, k)
    hd = sp.spherical_jn(l, k, True) + 1j * sp.spherical_yn(l, k, True)
    return 0.5 + 0.5j * k * k * (j * hd + jd * h) + eta * k * j * h


@pytest.mark.parametrize("l", [0, 1, 3])
def test_compiled_matvec_sphere_spectrum(l):
    errs = []
    for n in (1000, 4000):
        s = synth.unit_sphere(n, k=2.0, eta=1.5)
        v = np.sqrt(s.weights) * sp.eval_legendre(l, s.points[2])
        lam = _cfie_eigenvalue(l, 2.0, 1.5)
        av = cmatvec.matvec(s.points, s.normals, s.weights, 2.0, 1.5, v)
        errs.append(np.linalg.norm(av - lam * v) / np.linalg.norm(v))
    assert errs[1] < 0.04 and errs[1] < 0.75 * errs[0]


def test_compiled_matvec_adjoint_identity_and_dense_agreement():
    s = synth.graded_ellipsoid(1500, seed=5)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    v = rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)
    au = cmatvec.matvec(s.points, s.normals, s.weights, s.k, s.eta, u)
    ahv = cmatvec.matvec(s.points, s.normals, s.weights, s.k, s.eta, v, adjoint=True)
    assert abs(np.vdot(v, au) - np.vdot(ahv, u)) <= 1e-13 * np.linalg.norm(au) * np.linalg.norm(v)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    assert np.linalg.norm(au - a @ u) <= 1e-14 * np.linalg.norm(a @ u) * 10
    rows = np.array([0, 17, 1499, 600])
    assert np.array_equal(cmatvec.matvec_rows(s.points, s.normals, s.weights, s.k, s.eta, u, rows), au[rows])


@pytest.mark.parametrize("restart", [400, 7])
def test_gmres_matches_dense_lu(restart):
    s = synth.graded_ellipsoid(2000, seed=2)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    xs = dense.DenseLU(a).solve(b)
    x, rel, its = gmres.gmres(lambda v: a @ v, b, tol=1e-13, restart=restart, maxit=3000)
    assert rel <= 1e-13
    assert np.isclose(rel, np.linalg.norm(b - a @ x) / np.linalg.norm(b), rtol=1e-6, atol=0)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-12
    assert its > 10  # a genuine iteration, not a lucky first step


def test_gmres_adjoint_with_compiled_matvec():
    s = synth.unit_sphere(1500)
    a = dense.system_matrix(s.points, s.normals, s.weights, s.k, s.eta)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    ys = dense.DenseLU(a).solve_adjoint(b)
    y, rel, _ = gmres.gmres(lambda v: cmatvec.matvec(s.points, s.normals, s.weights, s.k, s.eta, v, adjoint=True),
                            b, tol=1e-13)
    assert rel <= 1e-13 and np.linalg.norm(y - ys) / np.linalg.norm(ys) <= 1e-12


def test_gmres_zero_rhs():
    x, rel, its = gmres.gmres(lambda v: 2.0 * v, np.zeros(5, complex))
    assert np.all(x == 0) and rel == 0.0 and its == 0
