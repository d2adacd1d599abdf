"""Seeded synthetic workloads: surface samples, weights, normals and Dirichlet data.

This module is the only code shared by the CPU oracle and the GPU path. It holds
no step of the factorization or of the solve: it only produces inputs (points on
a surface, outward normals, smooth quadrature weights, boundary data), each from
a seeded ``numpy.random.default_rng`` or a closed-form lattice.

The paper's own geometries (a wiggly torus discretized with locally corrected
quadrature on triangles, a model aircraft mesh; Section 6) cannot be reproduced
without those meshes and quadrature tables, so synthetic surfaces with plain
Nystrom weights stand in for them: the unit sphere, a strongly graded ellipsoid,
a bumpy sphere, and batches of independent scatterers.

All arrays are float64. Points and normals are returned structure-of-arrays,
shape (3, n); weights have shape (n,).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Surface",
    "fibonacci_sphere_dirs",
    "unit_sphere",
    "graded_ellipsoid",
    "bumpy_sphere",
    "scatterer_batch",
    "point_source_data",
    "plane_wave_data",
    "exterior_targets",
    "near_corrections",
    "by_name",
]


@dataclass
class Surface:
    """A sampled closed surface: points x (3, n), outward normals (3, n), weights (n,)."""

    points: np.ndarray
    normals: np.ndarray
    weights: np.ndarray
    k: float
    eta: float
    eps: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[1])


def fibonacci_sphere_dirs(n: int) -> np.ndarray:
    """Fibonacci lattice on the unit sphere: z_i = 1 - (2i+1)/n, phi_i = i*pi*(3 - sqrt 5).

    Returns (3, n) float64 unit vectors.
    """
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z])


def unit_sphere(n: int = 3000, k: float = 1.0, eta: float = 1.0, eps: float = 1e-6) -> Surface:
    """Unit sphere, Fibonacci lattice, equal weights 4*pi/n, normals = points."""
    x = fibonacci_sphere_dirs(n)
    w = np.full(n, 4.0 * math.pi / n)
    return Surface(x, x.copy(), w, k, eta, eps, name=f"unit_sphere_n{n}")


def _ellipsoid_area_density_integral(axes, density, nth=240, nph=480):
    """Integral of density over the ellipsoid surface (x/a)^2+(y/b)^2+(z/c)^2 = 1.

    Gauss-Legendre in the polar angle (three panels, graded towards the +z tip) and
    the periodic trapezoid rule in azimuth.
    """
    a, b, c = axes
    total = 0.0
    ph = (np.arange(nph) + 0.5) * (2.0 * math.pi / nph)
    for lo, hi in ((0.0, 0.5), (0.5, 1.5), (1.5, math.pi)):
        t, tw = np.polynomial.legendre.leggauss(nth)
        th = 0.5 * (hi - lo) * t + 0.5 * (hi + lo)
        tw = 0.5 * (hi - lo) * tw
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        st, ct = np.sin(TH), np.cos(TH)
        sp, cp = np.sin(PH), np.cos(PH)
        x = np.stack([a * st * cp, b * st * sp, c * ct])
        jac = st * np.sqrt((b * c * st * cp) ** 2 + (a * c * st * sp) ** 2 + (a * b * ct) ** 2)
        f = density(x.reshape(3, -1)).reshape(jac.shape) * jac
        total += float(np.sum(f * tw[:, None]) * (2.0 * math.pi / nph))
    return total


def _uniform_sphere(rng, m):
    g = rng.standard_normal((3, m))
    return g / np.linalg.norm(g, axis=0)


def graded_ellipsoid(
    n: int = 50_000,
    axes=(1.0, 2.0, 4.0),
    seed: int = 2,
    k: float = 2.0 * math.pi,
    eta: float | None = None,
    eps: float = 1e-6,
    peak: float = 20.0,
    width2: float = 0.05,
) -> Surface:
    """Ellipsoid with points graded towards the +z tip.

    Area-uniform proposals: u uniform on the unit sphere, mapped to x = diag(axes) u and
    accepted with probability J(u)/J_max, J(u) = abc*|diag(axes)^-1 u| (the area
    element of the map). A second acceptance with probability rho(x)/(1+peak) gives
    points with surface density proportional to rho(x) = 1 + peak*exp(-|x - tip|^2/width2).
    Weights w_i = Z/(n rho(x_i)) with Z the surface integral of rho, so that sum w_i f(x_i)
    estimates the surface integral of f.
    """
    if eta is None:
        eta = k
    a, b, c = (float(v) for v in axes)
    lam = np.array([a, b, c])
    tip = np.array([0.0, 0.0, c])
    rng = np.random.default_rng(seed)

    def rho(x):
        d2 = np.sum((x - tip[:, None]) ** 2, axis=0)
        return 1.0 + peak * np.exp(-d2 / width2)

    jmax = a * b * c / min(a, b, c)
    pts, nrm = [], []
    have = 0
    while have < n:
        m = 4 * (n - have) + 1024
        u = _uniform_sphere(rng, m)
        li = u / lam[:, None]
        ln = np.linalg.norm(li, axis=0)
        jac = a * b * c * ln
        keep = rng.random(m) < jac / jmax
        u, li, ln = u[:, keep], li[:, keep], ln[keep]
        x = lam[:, None] * u
        keep2 = rng.random(x.shape[1]) < rho(x) / (1.0 + peak)
        x, li, ln = x[:, keep2], li[:, keep2], ln[keep2]
        pts.append(x)
        nrm.append(li / ln)
        have += x.shape[1]
    x = np.concatenate(pts, axis=1)[:, :n]
    nv = np.concatenate(nrm, axis=1)[:, :n]
    z = _ellipsoid_area_density_integral((a, b, c), rho)
    w = z / (n * rho(x))
    return Surface(np.ascontiguousarray(x), np.ascontiguousarray(nv), w, k, eta, eps,
                   name=f"graded_ellipsoid_n{n}", meta={"seed": seed, "Z": z, "axes": (a, b, c)})


def bumpy_sphere(
    n: int = 100_000,
    nbumps: int = 200,
    seed: int = 4,
    k: float = 5.0,
    eta: float | None = None,
    eps: float = 1e-6,
) -> Surface:
    """Unit sphere carrying seeded Gaussian bumps, sampled adaptively.

    r(u) = 1 + sum_j h_j exp(-|u - c_j|^2 / (2 s_j^2)) with centres c_j uniform on the
    sphere, heights h_j ~ U[0.05, 0.2], widths s_j ~ U[0.01, 0.2]. Points have density
    proportional to ell(u)^-2 per unit area, ell(u)^-2 = 0.2^-2 + sum_j s_j^-2
    exp(-|u - c_j|^2 / (2 (2 s_j)^2)), so spacing follows the local bump width.

    Sampling: on the unit sphere |u - c|^2 = 2 - 2 u.c, so ell^-2 is a constant plus a sum of
    von Mises-Fisher densities with concentrations 1/(4 s_j^2); parameters u are drawn
    exactly from that mixture and accepted with probability J(u)/J_max, J the area element
    of the radial map x = r(u) u. Normals come from the gradient of |x| - r(x/|x|);
    weights are Z/(n ell^-2(u)) with Z = int ell^-2 dA estimated from the proposals.
    """
    if eta is None:
        eta = k
    rng = np.random.default_rng(seed)
    cen = _uniform_sphere(rng, nbumps)
    h = rng.uniform(0.05, 0.2, nbumps)
    s = rng.uniform(0.01, 0.2, nbumps)
    kap = 1.0 / (4.0 * s * s)
    base = 0.2 ** -2
    # mixture masses over the unit sphere: constant part and each vMF part
    m_base = base * 4.0 * math.pi
    m_bump = (s ** -2) * 2.0 * math.pi * (-np.expm1(-2.0 * kap)) / kap
    z_rho = m_base + m_bump.sum()
    probs = np.concatenate([[m_base], m_bump]) / z_rho

    def draw(m):
        comp = rng.choice(nbumps + 1, size=m, p=probs)
        u = _uniform_sphere(rng, m)
        sel = np.nonzero(comp > 0)[0]
        if sel.size:
            c = cen[:, comp[sel] - 1]
            kk = kap[comp[sel] - 1]
            xi = rng.random(sel.size)
            wcos = 1.0 + np.log(xi + (1.0 - xi) * np.exp(-2.0 * kk)) / kk
            wcos = np.clip(wcos, -1.0, 1.0)
            # unit tangent direction at c, uniform in angle
            t = _uniform_sphere(rng, sel.size)
            t = t - c * np.sum(t * c, axis=0)
            t = t / np.linalg.norm(t, axis=0)
            u[:, sel] = wcos * c + np.sqrt(np.maximum(0.0, 1.0 - wcos * wcos)) * t
        return u

    def surface(u):
        dots = cen.T @ u  # (nb, m)
        e = h[:, None] * np.exp((dots - 1.0) / (s * s)[:, None])
        r = 1.0 + e.sum(axis=0)
        g = cen @ (e / (s * s)[:, None])  # ambient gradient of r(u/|u|) at |u| = 1
        g = g - u * np.sum(g * u, axis=0)
        jac = r * np.sqrt(r * r + np.sum(g * g, axis=0))
        rho = base + np.sum((s ** -2)[:, None] * np.exp(kap[:, None] * (dots - 1.0)), axis=0)
        return jac, r, g, rho

    surface_one = surface
    if nbumps > 500:
        # many bumps: the (bumps x samples) arrays are evaluated in fixed column blocks on
        # host threads (same values for any thread count)
        import concurrent.futures as cf

        def surface(u):
            blk = 16384
            parts = [u[:, i:i + blk] for i in range(0, u.shape[1], blk)]
            with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                res = list(ex.map(surface_one, parts))
            return (np.concatenate([q[0] for q in res]), np.concatenate([q[1] for q in res]),
                    np.concatenate([q[2] for q in res], axis=1), np.concatenate([q[3] for q in res]))

    pts, nrm, dv, jsum, jcount = [], [], [], 0.0, 0
    probe = draw(100_000)
    jmax = 1.25 * float(surface(probe)[0].max())
    have = 0
    while have < n:
        m = min(200_000, int(1.6 * (n - have)) + 4096)
        u = draw(m)
        ja, r, g, rho = surface(u)
        jsum += float(ja.sum())
        jcount += m
        keep = rng.random(m) < ja / jmax
        u, r, g, rho = u[:, keep], r[keep], g[:, keep], rho[keep]
        x = r * u
        nv = u - g / r  # gradient of |x| - r(x/|x|) at |x| = r
        nv = nv / np.linalg.norm(nv, axis=0)
        pts.append(x)
        nrm.append(nv)
        dv.append(rho)
        have += x.shape[1]
    x = np.concatenate(pts, axis=1)[:, :n]
    nv = np.concatenate(nrm, axis=1)[:, :n]
    dd = np.concatenate(dv)[:n]
    z_est = z_rho * jsum / jcount  # int ell^-2 J du = Z_rho E_mixture[J]
    w = z_est / (n * dd)
    return Surface(np.ascontiguousarray(x), np.ascontiguousarray(nv), w, k, eta, eps,
                   name=f"bumpy_sphere_n{n}_b{nbumps}", meta={"seed": seed, "Z": z_est})


def scatterer_batch(count: int = 64, seed: int = 3, nmin: int = 2000, nmax: int = 20000,
                    eps: float = 1e-5) -> list[Surface]:
    """Independent spheres/ellipsoids with seeded axes in [0.5, 3], sizes in [nmin, nmax],
    wavenumbers k ~ U[1, 8] and eta = k. Fibonacci lattice mapped by the axes; weights
    (4*pi/N) times the area element of the map."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        sphere = rng.random() < 0.5
        if sphere:
            r = rng.uniform(0.5, 3.0)
            ax = np.array([r, r, r])
        else:
            ax = rng.uniform(0.5, 3.0, 3)
        n = int(rng.integers(nmin, nmax + 1))
        k = float(rng.uniform(1.0, 8.0))
        u = fibonacci_sphere_dirs(n)
        li = u / ax[:, None]
        ln = np.linalg.norm(li, axis=0)
        x = ax[:, None] * u
        w = (4.0 * math.pi / n) * float(np.prod(ax)) * ln
        out.append(Surface(x, li / ln, w, k, k, eps, name=f"scatterer{s}",
                           meta={"axes": tuple(ax.tolist()), "sphere": bool(sphere)}))
    return out


def point_source_data(points: np.ndarray, k: float, src=(0.1, 0.2, 0.3)) -> np.ndarray:
    """Dirichlet data of a point source inside the surface: e^{ik r}/(4 pi r), r = |x - src|."""
    d = points - np.asarray(src, dtype=np.float64)[:, None]
    r = np.sqrt(np.sum(d * d, axis=0))
    return np.exp(1j * k * r) / (4.0 * math.pi * r)


def plane_wave_data(points: np.ndarray, k: float, direction) -> np.ndarray:
    """Dirichlet data -exp(i k d.x) that cancels an incident plane wave along unit d."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return -np.exp(1j * k * (d @ points))


def near_corrections(points: np.ndarray, seed: int = 0, kref: int = 8, radius_factor: float = 2.5,
                     maxnb: int = 24, amp: float = 0.3, long_frac: float = 0.0, long_factor: float = 0.0,
                     long_max: int = 8):
    """Synthetic locally corrected quadrature: target-dependent weight factors for near pairs.

    For target i the quadrature weight of source j becomes w_j (1 + alpha_ij) for the listed
    pairs (a stand-in for the corrected near-field weights of a high-order rule, which are
    not available here). Pairs: the sources within radius_factor times the distance to the
    kref-th nearest neighbour of x_i (at most maxnb, nearest first, i itself excluded); for a
    fraction long_frac of the targets also up to long_max sources at distances in
    (that radius, long_factor times the kref-th neighbour distance], so that some corrections
    reach beyond a box's near field.
    alpha_ij ~ U[-amp, amp], seeded.

    Returns (row_ptr (n + 1), col (nnz), alpha (nnz)): CSR by target, columns ascending.
    """
    from scipy.spatial import cKDTree

    x = np.ascontiguousarray(np.asarray(points, dtype=np.float64).T)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    tree = cKDTree(x)
    dref, _ = tree.query(x, k=min(kref + 1, n))
    h = dref[:, -1] if dref.ndim == 2 else dref
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        r0 = radius_factor * h[i]
        near = np.asarray(tree.query_ball_point(x[i], r0), dtype=np.int64)
        near = near[near != i]
        if near.size > maxnb:
            dist = np.linalg.norm(x[near] - x[i], axis=1)
            near = near[np.argsort(dist, kind="stable")[:maxnb]]
        far = np.zeros(0, dtype=np.int64)
        if long_frac > 0.0 and rng.random() < long_frac:
            cand = np.asarray(tree.query_ball_point(x[i], long_factor * h[i]), dtype=np.int64)
            cand = cand[np.linalg.norm(x[cand] - x[i], axis=1) > r0]
            if cand.size:
                far = rng.choice(cand, size=min(long_max, cand.size), replace=False)
        c = np.unique(np.concatenate([near, far]))
        cols.append(c)
        vals.append(rng.uniform(-amp, amp, c.size))
        row_ptr[i + 1] = row_ptr[i] + c.size
    return row_ptr, np.concatenate(cols) if cols else np.zeros(0, np.int64), \
        np.concatenate(vals) if vals else np.zeros(0)


def exterior_targets(m: int = 50, seed: int = 0, rmin: float = 1.5, rmax: float = 3.0) -> np.ndarray:
    """Seeded targets outside the unit sphere: uniform directions, radius ~ U[rmin, rmax]."""
    rng = np.random.default_rng(seed)
    u = _uniform_sphere(rng, m)
    return u * rng.uniform(rmin, rmax, m)[None, :]


def by_name(name: str, **kw) -> Surface:
    """Named workloads: 'sphere3k' (n=3000, k=eta=1, eps=1e-6) and
    'ellipsoid50k' (n=50000 graded ellipsoid, k=2 pi, eta=k, eps=1e-6); sizes may be overridden."""
    if name == "sphere3k":
        return unit_sphere(kw.get("n", 3000), kw.get("k", 1.0), kw.get("eta", 1.0), kw.get("eps", 1e-6))
    if name == "ellipsoid50k":
        return graded_ellipsoid(kw.get("n", 50_000), seed=kw.get("seed", 2), k=kw.get("k", 2 * math.pi),
                                eps=kw.get("eps", 1e-6))
    if name == "bumpy100k":
        return bumpy_sphere(kw.get("n", 100_000), kw.get("nbumps", 200), seed=kw.get("seed", 4),
                            k=kw.get("k", 5.0), eps=kw.get("eps", 1e-6))
    raise KeyError(name)
