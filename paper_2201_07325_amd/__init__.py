"""MI355X (gfx950) FMM-LU: recursive strong skeletonization of the Helmholtz CFIE.

Thin ctypes binding of the C ABI declared in include/fmmlu.h. Every step of the
factorization and of the solves runs in the HIP library libfmmlu.so; this module only
marshals arguments. PyTorch provides device memory and the current HIP stream.

The library is required: importing works without it, but every call raises
RuntimeError if libfmmlu.so has not been built (python -m paper_2201_07325_amd.build).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import re
import weakref

import numpy as np

__all__ = ["lib", "Tree", "Factor", "kernel_block", "FmmluError", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmmlu.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fmmlu.h")

ENOCONV = -5
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR", -5: "ENOCONV", -6: "ESTATE"}


class FmmluError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.code = STATUS.get(status, str(status))


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("proxy_radius", C.c_double), ("proxy_min_points", C.c_int32),
                ("precision", C.c_int32), ("device_mem_cap", C.c_int64), ("verbose", C.c_int32),
                ("profile", C.c_int32), ("id_route", C.c_int32), ("test_zero_pivot_block", C.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("corr_row_ptr", C.c_void_p), ("corr_col", C.c_void_p), ("corr_a", C.c_void_p),
                ("gemm_autotune", C.c_int32), ("pchol_blocks", C.c_int32), ("reserved", C.c_int32 * 2)]


def _torch_alloc(nbytes, stream, ctx):
    """Device memory for the library from PyTorch's caching allocator (NULL on failure)."""
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=torch.cuda.current_device(),
                                                  stream=int(stream or 0))
    except Exception:  # reported by the library as FMMLU_ENOMEM
        return None


def _torch_free(ptr, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept alive for the life of the process: the library may call them until a factor is destroyed
_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)


def _set_allocator(o, allocator):
    if allocator == "torch":
        o.alloc, o.free, o.alloc_ctx = _TORCH_ALLOC, _TORCH_FREE, None
    elif allocator not in (None, "library"):
        raise ValueError("allocator must be 'torch' or 'library'")


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n0", C.c_int64), ("nlevels", C.c_int32),
                ("nboxes_factored", C.c_int32), ("factor_bytes", C.c_int64), ("peak_bytes", C.c_int64),
                ("max_rank", C.c_int32), ("max_block", C.c_int32), ("t_tree", C.c_double),
                ("t_factor", C.c_double), ("flops_id", C.c_double), ("flops_elim", C.c_double),
                ("flops_schur", C.c_double), ("flops_top", C.c_double), ("bytes_tiles", C.c_double),
                ("precision", C.c_int32), ("nspill", C.c_int32), ("reserved", C.c_int32 * 6)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None
# Factor and FactorBatch objects that own a library handle (borrowed views excluded)
_live = weakref.WeakSet()
P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
D = C.c_double
PD = C.POINTER(C.c_double)


def lib():
    """Load libfmmlu.so (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2201_07325_amd.build")
    L = C.CDLL(LIB_PATH)
    sig = {
        "fmmlu_default_opts": (I32, [C.POINTER(Opts)]),
        "fmmlu_build_tree": (I32, [PD, I64, I32, C.POINTER(P)]),
        "fmmlu_tree_info": (I32, [P, C.POINTER(I64), C.POINTER(I32), C.POINTER(I64)]),
        "fmmlu_tree_export": (I32, [P, P, P, P, P, P]),
        "fmmlu_tree_destroy": (None, [P]),
        "fmmlu_factor": (I32, [P, PD, PD, PD, D, D, C.POINTER(Opts), P, C.POINTER(P)]),
        "fmmlu_solve": (I32, [P, P, P, I64, P]),
        "fmmlu_solve_adjoint": (I32, [P, P, P, I64, P]),
        "fmmlu_matvec": (I32, [P, I32, P, P, P]),
        "fmmlu_matvec_noalloc": (I32, [P, I32, P, P, P]),
        "fmmlu_solve_refined": (I32, [P, P, P, I32, D, I32, C.POINTER(I32), PD, P]),
        "fmmlu_farfield": (I32, [P, P, I64, I32, P, P, P]),
        "fmmlu_dense_inverse": (I32, [P, I64, I64, P, P]),
        "fmmlu_set_solve_graph": (I32, [P, I32]),
        "fmmlu_factor_batch": (I32, [I32, P, P, P, P, P, P, P, I32, P]),
        "fmmlu_batch_info": (I32, [P, C.POINTER(I32), P]),
        "fmmlu_batch_factor": (I32, [P, I32, P]),
        "fmmlu_batch_solve": (I32, [P, P, P, I32, P]),
        "fmmlu_batch_destroy": (None, [P]),
        "fmmlu_factor_info": (I32, [P, C.POINTER(Info)]),
        "fmmlu_factor_boxes": (I32, [P, C.POINTER(I64), P, P, P, P, P]),
        "fmmlu_factor_box_data": (I32, [P, I64, P, P, P, P, P, P, P, P]),
        "fmmlu_factor_destroy": (None, [P]),
        "fmmlu_factor_profile": (I32, [P, P, P, P, P]),
        "fmmlu_kernel_block": (I32, [P, P, P, I64, D, D, P, I64, P, I64, P, P]),
        "fmmlu_proxy_block": (I32, [P, P, P, I64, D, D, P, I64, PD, D, I32, P, P]),
        "fmmlu_trim_caches": (I32, []),
        "fmmlu_gemm_tuning": (I32, [C.c_char_p, I64, C.POINTER(I64)]),
        "fmmlu_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/fmmlu.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fmmlu_[a-z_]+)\s*\(", txt)))


def _check(status):
    if status != 0:
        msg = lib().fmmlu_last_error().decode(errors="replace")
        raise FmmluError(status, msg)


def _soa(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim == 2 and a.shape[0] != 3 and a.shape[1] == 3:
        a = np.ascontiguousarray(a.T)
    if n is not None and a.size != 3 * n:
        raise ValueError("expected 3*n values")
    return a


def _ptr(a):
    return a.ctypes.data_as(PD)


class Tree:
    """Level-restricted adaptive octree (host). points: (3, n) float64."""

    def __init__(self, points, leaf_size=64):
        self.points = _soa(points)
        self.n = self.points.shape[-1] if self.points.ndim == 2 else self.points.size // 3
        h = P()
        _check(lib().fmmlu_build_tree(_ptr(self.points), self.n, int(leaf_size), C.byref(h)))
        self.h = h
        self.leaf_size = int(leaf_size)

    def info(self):
        nb, nl, nleaf = I64(), I32(), I64()
        _check(lib().fmmlu_tree_info(self.h, C.byref(nb), C.byref(nl), C.byref(nleaf)))
        return int(nb.value), int(nl.value), int(nleaf.value)

    def export(self):
        nb, nl, _ = self.info()
        level = np.zeros(nb, np.int32)
        coord = np.zeros((nb, 3), np.int32)
        npts = np.zeros(nb, np.int32)
        leaf = np.zeros(nb, np.int8)
        order = np.zeros(self.n, np.int64)
        _check(lib().fmmlu_tree_export(self.h, level.ctypes.data, coord.ctypes.data, npts.ctypes.data,
                                       leaf.ctypes.data, order.ctypes.data))
        return {"level": level, "coord": coord, "npts": npts, "is_leaf": leaf.astype(bool),
                "order": order, "nlevels": nl}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.fmmlu_tree_destroy(h)
            self.h = None


def _stream():
    import torch
    return P(torch.cuda.current_stream().cuda_stream)


def _dev_c128(x, n):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128):
        raise TypeError("expected a complex128 CUDA tensor")
    if x.shape[0] != n:
        raise ValueError(f"leading dimension {x.shape[0]} != n = {n}")
    return x


class Factor:
    """FMM-LU factorization of the scaled CFIE matrix on the current GPU.

    points, normals: (3, n) float64; weights: (n,) positive. Solves take and return
    complex128 CUDA tensors of shape (n,) or (n, nrhs) in the original point order.
    allocator: "torch" (default) takes every device block of the factorization from PyTorch's
    caching allocator (so torch.cuda.memory_allocated() counts it); "library" lets the
    library hipMalloc and cache its own blocks. test_zero_pivot_block >= 0 forces a zero pivot
    block at that eliminated box (failure-path testing). corrections: optional (row_ptr, col, a),
    CSR by target in the original point order: the entry (i, col) is multiplied by 1 + a
    (locally corrected quadrature weights w_ij = w_j (1 + a_ij)).
    """

    def __init__(self, points, normals, weights, k, eta, eps=1e-6, leaf_size=64, tree=None,
                 proxy_radius=2.5, proxy_min_points=64, precision=0, verbose=0, mem_cap=0, profile=False,
                 id_route=0, allocator="torch", test_zero_pivot_block=-1, corrections=None, gemm_autotune=1,
                 pchol_blocks=0):
        L = lib()
        self.points = _soa(points)
        self.n = self.points.size // 3
        self.normals = _soa(normals, self.n)
        self.weights = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        if self.weights.size != self.n:
            raise ValueError("weights must have n entries")
        self.k, self.eta, self.eps = float(k), float(eta), float(eps)
        self.tree = tree if tree is not None else Tree(self.points, leaf_size)
        o = Opts()
        _check(L.fmmlu_default_opts(C.byref(o)))
        o.eps = self.eps
        o.proxy_radius = float(proxy_radius)
        o.proxy_min_points = int(proxy_min_points)
        o.precision = int(precision)
        o.verbose = int(verbose)
        o.device_mem_cap = int(mem_cap)
        # True / 1: every kernel class; 2: the Schur-update class only
        o.profile = int(profile) if isinstance(profile, int) and not isinstance(profile, bool) else (1 if profile else 0)
        o.id_route = int(id_route)
        o.test_zero_pivot_block = int(test_zero_pivot_block)
        o.gemm_autotune = int(gemm_autotune)
        o.pchol_blocks = int(pchol_blocks)
        _set_allocator(o, allocator)
        keep = None
        if corrections is not None:
            rp, cc, ca = corrections
            keep = (np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(cc, dtype=np.int64),
                    np.ascontiguousarray(ca, dtype=np.float64))
            if keep[0].size != self.n + 1 or keep[1].size != keep[2].size or keep[1].size < keep[0][-1]:
                raise ValueError("corrections: row_ptr of n + 1 entries, col and a of row_ptr[n] entries")
            o.corr_row_ptr, o.corr_col, o.corr_a = keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data
        h = P()
        _check(L.fmmlu_factor(self.tree.h, _ptr(self.points), _ptr(self.normals), _ptr(self.weights),
                              self.k, self.eta, C.byref(o), _stream(), C.byref(h)))
        self.h = h
        _live.add(self)

    def _apply(self, fn, b, out=None):
        import torch
        b = _dev_c128(b, self.n)
        squeeze = b.dim() == 1
        bb = b.reshape(self.n, -1)
        nrhs = bb.shape[1]
        # column-major n x nrhs: column c contiguous
        bcol = bb.t().contiguous()
        x = torch.empty_like(bcol)
        _check(fn(self.h, P(bcol.data_ptr()), P(x.data_ptr()), nrhs, _stream()))
        x = x.t()
        return x.reshape(self.n) if squeeze else x.contiguous()

    def solve(self, b):
        """x = A_f^{-1} b."""
        return self._apply(lib().fmmlu_solve, b)

    def set_solve_graph(self, enable):
        """Replay solves from a captured HIP graph (default) or launch kernels one by one."""
        _check(lib().fmmlu_set_solve_graph(self.h, 1 if enable else 0))

    def solve_adjoint(self, b):
        """x = A_f^{-H} b."""
        return self._apply(lib().fmmlu_solve_adjoint, b)

    def solve_refined(self, b, adjoint=False, tol=1e-12, maxit=100, raise_on_fail=True):
        """Float64 FGMRES on A~ (adjoint: A~^H) preconditioned by the factored inverse.

        Returns (x, iterations, relative residual). With raise_on_fail False a run that
        stops at maxit returns its last iterate instead of raising FmmluError."""
        import torch
        b = _dev_c128(b, self.n).contiguous()
        if b.dim() != 1:
            raise ValueError("solve_refined takes one right-hand side")
        x = torch.empty_like(b)
        it = I32()
        rr = C.c_double()
        st = lib().fmmlu_solve_refined(self.h, P(b.data_ptr()), P(x.data_ptr()), 1 if adjoint else 0,
                                       float(tol), int(maxit), C.byref(it), C.byref(rr), _stream())
        if st != 0 and not (st == ENOCONV and not raise_on_fail):
            _check(st)
        return x, int(it.value), float(rr.value)

    def farfield(self, dirs, v, op=0):
        """Far-field pattern operator: op 0 C v, 1 C^H v, 2 (dC/dk) v, 3 (dC/deta) v.

        dirs: (3, ndir) float64 unit directions (CUDA tensor or host array)."""
        import torch
        d = torch.as_tensor(dirs, dtype=torch.float64).to("cuda").contiguous()
        if d.dim() != 2 or d.shape[0] != 3:
            raise ValueError("dirs must have shape (3, ndir)")
        ndir = d.shape[1]
        if op == 1:
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.complex128) or v.shape != (ndir,):
                raise ValueError("op 1 takes a complex128 CUDA vector of length ndir")
            out = torch.empty(self.n, dtype=torch.complex128, device=v.device)
        else:
            v = _dev_c128(v, self.n)
            out = torch.empty(ndir, dtype=torch.complex128, device=v.device)
        v = v.contiguous()
        _check(lib().fmmlu_farfield(self.h, P(d.data_ptr()), ndir, int(op), P(v.data_ptr()), P(out.data_ptr()),
                                    _stream()))
        return out

    def matvec(self, x, op=0):
        """Exact float64 product: op 0 A~, 1 A~^H, 2 dA~/dk, 3 dA~/deta."""
        import torch
        x = _dev_c128(x, self.n).contiguous()
        y = torch.empty_like(x)
        _check(lib().fmmlu_matvec(self.h, int(op), P(x.data_ptr()), P(y.data_ptr()), _stream()))
        return y

    def info(self):
        inf = Info()
        _check(lib().fmmlu_factor_info(self.h, C.byref(inf)))
        return inf.as_dict()

    KCLASSES = ["assemble", "id_matrix", "householder_qr", "pivoted_qr", "elimination", "pivot_inverse",
                "schur_update", "top_block"]

    def profile(self):
        """Per kernel class: GPU ms (HIP events), brackets, algorithmic flops and bytes."""
        nk = len(self.KCLASSES)
        ms = np.zeros(nk)
        la = np.zeros(nk, np.int64)
        fl = np.zeros(nk)
        by = np.zeros(nk)
        _check(lib().fmmlu_factor_profile(self.h, ms.ctypes.data, la.ctypes.data, fl.ctypes.data,
                                          by.ctypes.data))
        return {k: {"ms": float(ms[i]), "launches": int(la[i]), "flops": float(fl[i]), "bytes": float(by[i])}
                for i, k in enumerate(self.KCLASSES)}

    def boxes(self):
        cnt = I64()
        _check(lib().fmmlu_factor_boxes(self.h, C.byref(cnt), None, None, None, None, None))
        c = int(cnt.value)
        level = np.zeros(c, np.int32)
        coord = np.zeros((c, 3), np.int32)
        m = np.zeros(c, np.int32)
        s = np.zeros(c, np.int32)
        _check(lib().fmmlu_factor_boxes(self.h, C.byref(cnt), level.ctypes.data, coord.ctypes.data,
                                        m.ctypes.data, s.ctypes.data, None))
        skel = np.zeros(int(s.sum()), np.int64)
        _check(lib().fmmlu_factor_boxes(self.h, C.byref(cnt), None, None, None, None, skel.ctypes.data))
        return {"level": level, "coord": coord, "m": m, "s": s, "skel": skel}

    def box_data(self, rec):
        """Factors of record rec (elimination order) on the host: R, S, SN as original point
        indices (R, S in the ID's pivot order), T (s x r), Xi = X_RR^{-1} (r x r),
        L ((s + n_N) x r) and U ((r x (s + n_N)), complex128."""
        L_ = lib()
        sz = np.zeros(3, np.int32)
        _check(L_.fmmlu_factor_box_data(self.h, int(rec), sz.ctypes.data, None, None, None, None, None, None,
                                        None))
        r, s, nsn = (int(v) for v in sz)
        R = np.zeros(r, np.int64)
        S = np.zeros(s, np.int64)
        SN = np.zeros(nsn, np.int64)
        T = np.zeros((r, s), np.complex128)      # column-major s x r == row-major r x s
        Xi = np.zeros((r, r), np.complex128)
        Lt = np.zeros((r, nsn), np.complex128)
        UT = np.zeros((r, nsn), np.complex128)
        _check(L_.fmmlu_factor_box_data(self.h, int(rec), sz.ctypes.data, R.ctypes.data, S.ctypes.data,
                                        SN.ctypes.data, T.ctypes.data, Xi.ctypes.data, Lt.ctypes.data,
                                        UT.ctypes.data))
        return {"R": R, "S": S, "SN": SN, "T": T.T.copy(), "Xi": Xi.T.copy(), "L": Lt.T.copy(), "U": UT}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None and getattr(self, "_owner", None) is None:
            _lib.fmmlu_factor_destroy(h)
        self.h = None


def kernel_block(points, normals, weights, k, eta, rows, cols):
    """A~[rows, cols] generated on the device; returns a complex128 CUDA tensor (nr, nc)."""
    import torch
    pts = torch.as_tensor(_soa(points)).reshape(-1).cuda()
    n = pts.numel() // 3
    nrm = torch.as_tensor(_soa(normals, n)).reshape(-1).cuda()
    w = torch.as_tensor(np.asarray(weights, np.float64)).cuda()
    r = torch.as_tensor(np.asarray(rows, np.int64)).cuda()
    c = torch.as_tensor(np.asarray(cols, np.int64)).cuda()
    out = torch.empty((c.numel(), r.numel()), dtype=torch.complex128, device="cuda")
    _check(lib().fmmlu_kernel_block(P(pts.data_ptr()), P(nrm.data_ptr()), P(w.data_ptr()), n, float(k),
                                    float(eta), P(r.data_ptr()), r.numel(), P(c.data_ptr()), c.numel(),
                                    P(out.data_ptr()), _stream()))
    return out.t()


def proxy_block(points, normals, weights, k, eta, dofs, centre, radius, ngamma):
    """Proxy rows of the ID matrix generated on the device: a complex128 CUDA tensor
    (2 ngamma, len(dofs)), outgoing rows first, then incoming rows."""
    import torch
    pts = torch.as_tensor(_soa(points)).cuda()
    n = pts.numel() // 3
    nrm = torch.as_tensor(_soa(normals, n)).cuda()
    w = torch.as_tensor(np.ascontiguousarray(weights, dtype=np.float64)).cuda()
    d = torch.as_tensor(np.asarray(dofs, np.int64)).cuda()
    c = np.ascontiguousarray(centre, dtype=np.float64)
    out = torch.empty((d.numel(), 2 * int(ngamma)), dtype=torch.complex128, device="cuda")
    _check(lib().fmmlu_proxy_block(P(pts.data_ptr()), P(nrm.data_ptr()), P(w.data_ptr()), n, float(k),
                                   float(eta), P(d.data_ptr()), d.numel(), _ptr(c), float(radius), int(ngamma),
                                   P(out.data_ptr()), _stream()))
    return out.t()


def trim_caches():
    """Free the device and pinned host memory that released factorizations keep for reuse
    by later ones (call between factorizations)."""
    _check(lib().fmmlu_trim_caches())


def gemm_tuning():
    """The GEMM autotuner's table for the current device (dict: the kernel chosen per use and
    K bucket, and each candidate's measured milliseconds), or None before any factorization
    has tuned it."""
    import json
    need = I64(0)
    st = lib().fmmlu_gemm_tuning(None, 0, C.byref(need))
    if st != 0:
        return None
    buf = C.create_string_buffer(int(need.value))
    _check(lib().fmmlu_gemm_tuning(buf, need.value, None))
    return json.loads(buf.value.decode())


def release_all():
    """Destroy every factorization and batch this process still holds, then free the reuse
    caches. Registered with atexit, so that the library makes its last HIP calls while the
    interpreter is still running, before the runtime and any attached tools shut down."""
    if _lib is None:
        return
    for obj in list(_live):
        obj.__del__()
    _live.clear()
    _lib.fmmlu_trim_caches()


atexit.register(release_all)


def dense_inverse(a):
    """Inverses of a batch of complex128 CUDA matrices a (count, n, n) with the library's
    blocked Gauss-Jordan (the routine used for pivot and top blocks)."""
    import torch
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.complex128):
        raise TypeError("expected a complex128 CUDA tensor")
    squeeze = a.dim() == 2
    a3 = a.reshape(-1, a.shape[-2], a.shape[-1])
    cnt, n, n2 = a3.shape
    if n != n2:
        raise ValueError("matrices must be square")
    # column-major storage: the transpose of each row-major matrix
    ac = a3.transpose(1, 2).contiguous()
    out = torch.empty_like(ac)
    _check(lib().fmmlu_dense_inverse(P(ac.data_ptr()), n, cnt, P(out.data_ptr()), _stream()))
    res = out.transpose(1, 2)
    return res[0] if squeeze else res


class FactorBatch:
    """Independent problems (e.g. many scatterers) factored concurrently on the current GPU.

    problems: sequence of (points, normals, weights, k, eta). Solves take and return one
    concatenated complex128 CUDA vector; problem i occupies offsets[i]:offsets[i+1].
    """

    def __init__(self, problems, eps=1e-6, leaf_size=64, nthreads=0, proxy_radius=2.5, proxy_min_points=64,
                 id_route=0, precision=0, allocator="torch"):
        L = lib()
        self.problems = []
        for pts, nrm, w, k, eta in problems:
            p = _soa(pts)
            n = p.size // 3
            self.problems.append((p, _soa(nrm, n), np.ascontiguousarray(np.asarray(w, dtype=np.float64)),
                                  float(k), float(eta)))
        cnt = len(self.problems)
        if cnt < 1:
            raise ValueError("empty batch")
        self.trees = [Tree(p[0], leaf_size) for p in self.problems]
        arr = lambda vals: (P * cnt)(*vals)
        trees = arr([t.h for t in self.trees])
        xyz = arr([p[0].ctypes.data for p in self.problems])
        nrm = arr([p[1].ctypes.data for p in self.problems])
        ws = arr([p[2].ctypes.data for p in self.problems])
        ks = (C.c_double * cnt)(*[p[3] for p in self.problems])
        etas = (C.c_double * cnt)(*[p[4] for p in self.problems])
        o = Opts()
        _check(L.fmmlu_default_opts(C.byref(o)))
        o.eps = float(eps)
        o.proxy_radius = float(proxy_radius)
        o.proxy_min_points = int(proxy_min_points)
        o.id_route = int(id_route)
        o.precision = int(precision)
        _set_allocator(o, allocator)
        h = P()
        _check(L.fmmlu_factor_batch(cnt, trees, xyz, nrm, ws, ks, etas, C.byref(o), int(nthreads), C.byref(h)))
        self.h = h
        _live.add(self)
        c = I32()
        off = np.zeros(cnt + 1, np.int64)
        _check(L.fmmlu_batch_info(self.h, C.byref(c), off.ctypes.data))
        self.count = int(c.value)
        self.offsets = off
        self.n = int(off[-1])

    def solve(self, b, adjoint=False):
        import torch
        b = _dev_c128(b, self.n).contiguous()
        x = torch.empty_like(b)
        _check(lib().fmmlu_batch_solve(self.h, P(b.data_ptr()), P(x.data_ptr()), 1 if adjoint else 0, _stream()))
        return x

    def factor(self, i):
        """Borrowed view of problem i's factorization (solve, matvec, info); the batch owns it."""
        h = P()
        _check(lib().fmmlu_batch_factor(self.h, int(i), C.byref(h)))
        f = Factor.__new__(Factor)
        p = self.problems[i]
        f.points, f.normals, f.weights, f.k, f.eta = p[0], p[1], p[2], p[3], p[4]
        f.n = p[0].size // 3
        f.h = h
        f._owner = self
        return f

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.fmmlu_batch_destroy(h)
            self.h = None

