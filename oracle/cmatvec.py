"""Compiled exact matvec with the scaled CFIE matrix (oracle; test infrastructure).

Thin ctypes loader for `matvec.c`: the same closed-form entries as `dense.system_matrix`
(Section 3, eqs. disc1, disc3, comb_ref), formed one at a time and summed in index order,
so that products with the full matrix at tens of thousands of unknowns are affordable.
The shared object is compiled with gcc and OpenMP, on first use if `build()` has not
already done it; IEEE arithmetic (no fast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "matvec.c")
LIB = os.path.join(HERE, "liboracle_matvec.so")
_lib = None


def build():
    """Compile matvec.c into liboracle_matvec.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp, "-lm"],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        lib.oracle_matvec.argtypes = [p, p, p, ctypes.c_int64, ctypes.c_double, ctypes.c_double, p, p,
                                      ctypes.c_int]
        lib.oracle_matvec_rows.argtypes = [p, p, p, ctypes.c_int64, ctypes.c_double, ctypes.c_double, p,
                                           p, ctypes.c_int64, p]
        _lib = lib
    return _lib


def _geom(x, nrm, w):
    x = np.ascontiguousarray(x, dtype=np.float64)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    sw = np.ascontiguousarray(np.sqrt(np.asarray(w, dtype=np.float64)))
    return x, nrm, sw


def matvec(x, nrm, w, k, eta, v, adjoint=False):
    """A~ v, or A~^H v with adjoint=True, for v of shape (n,)."""
    x, nrm, sw = _geom(x, nrm, w)
    n = x.shape[1]
    v = np.ascontiguousarray(v, dtype=np.complex128)
    assert v.shape == (n,)
    y = np.empty(n, dtype=np.complex128)
    _load().oracle_matvec(x.ctypes.data, nrm.ctypes.data, sw.ctypes.data, n, float(k), float(eta),
                          v.ctypes.data, y.ctypes.data, int(bool(adjoint)))
    return y


def matvec_rows(x, nrm, w, k, eta, v, rows):
    """(A~ v)[rows] without forming the other rows."""
    x, nrm, sw = _geom(x, nrm, w)
    n = x.shape[1]
    v = np.ascontiguousarray(v, dtype=np.complex128)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    assert v.shape == (n,) and rows.ndim == 1 and (rows.size == 0 or (rows.min() >= 0 and rows.max() < n))
    y = np.empty(rows.size, dtype=np.complex128)
    _load().oracle_matvec_rows(x.ctypes.data, nrm.ctypes.data, sw.ctypes.data, n, float(k), float(eta),
                               v.ctypes.data, rows.ctypes.data, rows.size, y.ctypes.data)
    return y
