"""Writes the reference solutions of the graded-ellipsoid workload (n = 50,000).

Calls only the oracle: the workload from `synth.graded_ellipsoid(50000, seed=2)`
(k = 2 pi, eta = k), right-hand side b = sqrt(w) times the field of a point source at
(0.1, 0.2, 0.3) (the interior-source test of Section 6.1), and

    x* = A~^{-1} b     and     y* = A~^{-H} b

by unpreconditioned float64 GMRES (oracle.gmres) with the exact compiled matvec
(oracle.cmatvec), each run until the true relative residual is <= 1e-13. Dense LU of
the 50,000 x 50,000 complex matrix (40 GB) is replaced by this iteration, whose error is
bounded by the condition number times the residual.

Output: ellipsoid50k_reference.npz beside this script (x, y, b's parameters, residuals,
iteration counts). Takes about an hour on eight cores:
    python tests/golden/make_ellipsoid50k_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cmatvec, gmres  # noqa: E402

OUT = os.path.join(HERE, "ellipsoid50k_reference.npz")
TOL = 1e-13


def main():
    s = synth.graded_ellipsoid(50_000, seed=2)
    b = np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)
    res = {}
    for name, adj in (("x", False), ("y", True)):
        t0 = time.time()

        def mv(v, adj=adj):
            return cmatvec.matvec(s.points, s.normals, s.weights, s.k, s.eta, v, adjoint=adj)

        def log(it, est):
            print(f"{name}: iteration {it}, residual estimate {est:.3e}, {time.time() - t0:.0f} s", flush=True)

        sol, rel, its = gmres.gmres(mv, b, tol=TOL, restart=400, maxit=1200, log=log)
        print(f"{name}: relres {rel:.3e} after {its} iterations, {time.time() - t0:.0f} s", flush=True)
        if rel > TOL:
            raise SystemExit(f"{name}: GMRES stopped at relres {rel:.3e} > {TOL}")
        res[name] = (sol, rel, its)
    np.savez(OUT, x=res["x"][0], y=res["y"][0], relres_x=res["x"][1], relres_y=res["y"][1],
             iterations_x=res["x"][2], iterations_y=res["y"][2], n=s.n, seed=2, k=s.k, eta=s.eta,
             source=np.array([0.1, 0.2, 0.3]), tol=TOL)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
