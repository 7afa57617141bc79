"""The allocation-free product hh_matvec_noalloc, called through the C ABI:
bit for bit the result of hh_matvec / hh_matvec_t on two calls in a row (the
second on a smaller matrix, so the shared scratch holds the first call's
larger contents), for one and several right-hand sides and both directions;
a product whose workspace exceeds the scratch is refused with HH_ENOTSUP."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(g, x, y, nrhs, trans):
    import torch
    from paper_2604_09147_amd import hh
    st = hh.lib().hh_matvec_noalloc(g._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                    nrhs, int(trans), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_noalloc_product_equals_the_allocating_product():
    torch = _torch()
    from paper_2604_09147_amd import HMatrix, hh
    rng = np.random.default_rng(61)
    big = HMatrix(rng.random((6000, 3)), W.INV_R, 1e-6, 1.5, -1, 64)
    small = HMatrix(rng.random((1500, 2)), W.LOG, 1e-8, 1.0, -1, 32)
    print("noalloc: handles of 6000 (3D) and 1500 (2D) points built", flush=True)
    for nrhs, trans in ((1, False), (1, True), (3, False), (3, True)):
        for g in (big, small):                  # the second call is the smaller one
            shape = (g.n,) if nrhs == 1 else (g.n, nrhs)
            x = torch.from_numpy(rng.standard_normal(shape)).cuda()
            ref = g.matvec_t(x) if trans else g.matvec(x)
            y = torch.full_like(x, float("nan"))
            assert _noalloc(g, x, y, nrhs, trans) == hh.HH_OK, hh.lib().hh_last_error()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (g.n, nrhs, trans)
    # more workspace than the scratch holds: refused before anything is queued
    nr = 2048
    x = torch.zeros((big.n, nr), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    assert _noalloc(big, x, y, nr, False) == hh.HH_ENOTSUP
    assert b"scratch" in hh.lib().hh_last_error()
    assert float(y.abs().sum()) == 0.0
    big.free()
    small.free()
