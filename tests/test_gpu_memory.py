"""Device memory and failure paths of the factorization, through the C ABI.

* With the caller's allocator (PyTorch's caching allocator, the binding's default) every
  device block of a factorization is visible to torch while the factor lives and is returned
  when it is destroyed; an allocator that runs dry is reported as FMMLU_ENOMEM and every block
  handed out before the failure is given back.
* peak_bytes counts factors, tile pools, scratch and upload buffers together; the device
  memory cap applies to that count: a cap at the measured peak passes, half of it fails with
  FMMLU_ENOMEM.
* A pivot block forced to zero from the host is reported as FMMLU_ESINGULAR, and the library
  keeps working afterwards.
* Run-to-run determinism: two factorizations of the same input, with either allocator, give
  bitwise identical skeletons and solutions.
"""
import ctypes as C
import gc

import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth

pytestmark = pytest.mark.gpu


def _surface():
    return synth.graded_ellipsoid(4000, seed=2, k=3.0)


def _factor(s, **kw):
    return fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6, leaf_size=32, **kw)


def _rhs(s):
    return torch.as_tensor(np.sqrt(s.weights) * synth.point_source_data(s.points, s.k)).cuda()


def test_torch_allocator_holds_and_returns_factor_memory():
    s = _surface()
    b = _rhs(s)
    torch.cuda.synchronize()
    gc.collect()
    base = torch.cuda.memory_allocated()
    f = _factor(s, allocator="torch")
    held = torch.cuda.memory_allocated() - base
    info = f.info()
    x = f.solve(b)
    torch.cuda.synchronize()
    print(f"factor_bytes {info['factor_bytes']}, held through torch {held}, peak {info['peak_bytes']}")
    assert held >= info["factor_bytes"] > 0
    assert info["peak_bytes"] >= held
    del f, x
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_runs_and_allocators_bitwise_identical():
    s = _surface()
    b = _rhs(s)
    outs = []
    for alloc in ("torch", "torch", "library"):
        f = _factor(s, allocator=alloc)
        outs.append((f.solve(b), f.solve_adjoint(b), f.boxes()["skel"], f.info()["n0"]))
        del f
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2]) and o[3] == outs[0][3]


def test_peak_bytes_and_memory_cap():
    s = _surface()
    fm.trim_caches()
    f = _factor(s, allocator="library")
    info = f.info()
    peak = int(info["peak_bytes"])
    print(f"peak {peak}, factor bytes {info['factor_bytes']}, tile bytes (all levels) {info['bytes_tiles']:.3e}")
    assert peak > info["factor_bytes"]
    del f
    for alloc in ("library", "torch"):
        g = _factor(s, allocator=alloc, mem_cap=peak)
        assert g.info()["peak_bytes"] <= peak
        del g
        with pytest.raises(fm.FmmluError) as e:
            _factor(s, allocator=alloc, mem_cap=peak // 2)
        assert e.value.code == "ENOMEM"


def test_allocator_failure_returns_enomem_and_gives_blocks_back():
    s = _surface()
    live = {}
    calls = {"n": 0}

    def alloc(nbytes, stream, ctx):
        calls["n"] += 1
        if calls["n"] > 6:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        live[p] = nbytes
        return p

    def free(ptr, stream, ctx):
        live.pop(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))

    af, ff = fm.ALLOC_FN(alloc), fm.FREE_FN(free)
    L = fm.lib()
    o = fm.Opts()
    L.fmmlu_default_opts(C.byref(o))
    o.alloc, o.free = af, ff
    t = fm.Tree(s.points, 32)
    h = C.c_void_p()
    pts, nrm, w = fm._soa(s.points), fm._soa(s.normals, s.n), np.ascontiguousarray(s.weights)
    rc = L.fmmlu_factor(t.h, fm._ptr(pts), fm._ptr(nrm), fm._ptr(w), s.k, s.eta, C.byref(o), fm._stream(),
                        C.byref(h))
    assert rc == -2, L.fmmlu_last_error().decode()
    assert calls["n"] == 7 and not live and not h.value


def test_zero_pivot_block_reports_esingular():
    s = _surface()
    with pytest.raises(fm.FmmluError) as e:
        _factor(s, test_zero_pivot_block=5)
    assert e.value.code == "ESINGULAR"
    f = _factor(s)
    x = f.solve(_rhs(s))
    assert torch.isfinite(torch.view_as_real(x)).all()
