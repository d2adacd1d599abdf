"""Allocation-free matvec (fmmlu_matvec_noalloc) against fmmlu_matvec, through the C ABI.

The allocation-free entry point runs the same kernels with its scratch in a static device
array, so its output must equal the allocating entry point's bitwise. Two calls in a row,
the second on a smaller problem (the array keeps the first call's contents), every op;
device memory reported free by the runtime must not change across the calls.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2201_07325_amd as fm
import synth

pytestmark = pytest.mark.gpu


def _noalloc(f, op, x, y):
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fm.lib().fmmlu_matvec_noalloc(f.h, int(op), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), st)
    assert rc == 0, fm.lib().fmmlu_last_error().decode()


def test_noalloc_matvec_matches_matvec_two_calls_shrinking():
    torch.cuda.set_device(0)
    big = synth.graded_ellipsoid(6000, seed=2)
    small = synth.unit_sphere(1500)
    fb = fm.Factor(big.points, big.normals, big.weights, big.k, big.eta, eps=1e-6)
    fs = fm.Factor(small.points, small.normals, small.weights, small.k, small.eta, eps=1e-6)
    rng = np.random.default_rng(7)
    xb = torch.as_tensor(rng.standard_normal(big.n) + 1j * rng.standard_normal(big.n)).cuda()
    xs = torch.as_tensor(rng.standard_normal(small.n) + 1j * rng.standard_normal(small.n)).cuda()
    refs = {(name, op): (f.matvec(x, op)) for name, f, x in (("big", fb, xb), ("small", fs, xs))
            for op in range(4)}
    outs = {(name, op): torch.full_like(x, complex(np.nan, np.nan)) for name, x in (("big", xb), ("small", xs))
            for op in range(4)}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for op in range(4):
        _noalloc(fb, op, xb, outs[("big", op)])    # first call: the larger problem
        _noalloc(fs, op, xs, outs[("small", op)])  # second call: smaller, over the first one's scratch
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for key, y in outs.items():
        ref = refs[key]
        assert torch.isfinite(torch.view_as_real(y)).all(), key
        assert torch.equal(y, ref), (key, float(torch.max(torch.abs(y - ref))))
    assert free1 == free0


def test_noalloc_rejects_bad_arguments():
    s = synth.unit_sphere(800)
    f = fm.Factor(s.points, s.normals, s.weights, s.k, s.eta, eps=1e-6)
    x = torch.zeros(s.n, dtype=torch.complex128, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = fm.lib()
    assert L.fmmlu_matvec_noalloc(f.h, 4, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr() + 16), st) == -1
    assert L.fmmlu_matvec_noalloc(f.h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), st) == -1
    assert L.fmmlu_matvec_noalloc(None, 0, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), st) == -6
