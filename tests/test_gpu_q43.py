"""GPU parity of q43 storage (the 8-bit row of the paper's format table, mask
bit 5 of the C header, bit 4 of the oracle) against the FP64 oracle.

Bars: structure (tree, partition, ranks, formats) bit for bit with the tie
rule; every stored q43 factor is an exact q43 value after its power-of-two
scale, the largest entry of each factor scaled into [64, 128] (Alg. 3 storage
with the scaling rule of the 16-bit formats); the kernel product within the
fp32-arithmetic bound of the fp64 product of its own exported factors
(1, several and many right-hand sides, both directions); the product within
tol / 10 of the oracle's and within 10 tol of the dense product. The oracle bar
is wider than the 1e-2 tol of the 16-bit tests: one entry that two correct
SVDs put on opposite sides of a q43 rounding boundary moves that block's
product by up to 2^-4 of its share, against 2^-11 for fp16."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import HH_FMT_Q43, compare_structure, exported_product, rel, within_kernel_bound

pytestmark = pytest.mark.gpu

GPU_MASK = 0x2F                 # fp64, fp32, fp16, bf16, q43
ORACLE_MASK = 0x1F


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _build(P, kind, tol, eta, leaf):
    from paper_2604_09147_amd import HMatrix
    g = HMatrix(P, kind, tol, eta, -1, leaf, mask=GPU_MASK)
    o = O.build(P, O.Kernel(kind), tol, eta, -1, leaf, mask=ORACLE_MASK)
    return g, o


def _check_stored_codes(g):
    bl = g.blocks()
    q43 = np.flatnonzero((bl["format"] == HH_FMT_Q43) & (bl["rank"] > 0))
    assert q43.size > 0
    for q in q43[:: max(1, q43.size // 200)]:
        A, B = g.block_factors(int(q))
        for F, e in ((A, int(bl["exp_u"][q])), (B, int(bl["exp_v"][q]))):
            s = np.ldexp(F, -e)
            assert np.array_equal(O.round_q43(s), s), q
            m = np.max(np.abs(s))
            assert 64.0 <= m <= 128.0, (q, m)


def _check_products(g, o, P, kind, tol, nrhs, trans, seed):
    torch = _torch()
    rng = np.random.default_rng(seed)
    shape = (P.shape[0],) if nrhs == 1 else (P.shape[0], nrhs)
    x = rng.standard_normal(shape)
    xd = torch.from_numpy(x).cuda()
    y = (g.matvec_t(xd) if trans else g.matvec(xd)).cpu().numpy()
    ye, bound = exported_product(g, x, trans)
    assert within_kernel_bound(y, ye, bound), rel(y, ye)
    yo = O.matvec_t(o, x) if trans else O.matvec(o, x)
    assert rel(y, yo) <= 0.1 * tol, rel(y, yo)
    k = O.Kernel(kind)
    yd = O.dense_matvec_t(P, k, x) if trans else O.dense_matvec(P, k, x)
    assert rel(y, yd) <= 10 * tol, rel(y, yd)


@pytest.mark.parametrize("kind,d,tol,eta", [
    (W.INV_R, 3, 1e-2, 1.5),            # mostly q43, some bf16
    (W.LOG, 2, 1e-2, 1.0),              # q43 and bf16, L = 4
    (W.INV_R, 3, 3e-3, 1.5)])           # mostly bf16, a few q43
def test_q43_storage_against_the_oracle(kind, d, tol, eta):
    rng = np.random.default_rng(kind * 10 + d + 7)
    P = rng.random((3001, d))
    g, o = _build(P, kind, tol, eta, 24)
    compare_structure(g, o)
    s = g.stats()
    assert s["blocks_by_format"][HH_FMT_Q43] > 0
    assert s["factor_bytes_by_format"][HH_FMT_Q43] > 0
    _check_stored_codes(g)
    for nrhs in (1, 5, 20, 40):
        for trans in (False, True):
            _check_products(g, o, P, kind, tol, nrhs, trans, seed=nrhs + 100 * trans)
    g.free()


def test_q43_batched_with_a_fixed_format_handle():
    # a batch of a q43 handle and a handle without q43 runs on the q43 kernels
    torch = _torch()
    from paper_2604_09147_amd import HMatrix, matvec_batch
    rng = np.random.default_rng(21)
    P1, P2 = rng.random((2500, 3)), rng.random((1800, 2))
    g1 = HMatrix(P1, W.INV_R, 1e-2, 1.5, -1, 24, mask=GPU_MASK)
    g2 = HMatrix(P2, W.LOG, 1e-6, 1.0, -1, 24)
    assert g1.stats()["blocks_by_format"][HH_FMT_Q43] > 0
    assert g2.stats()["blocks_by_format"][HH_FMT_Q43] == 0
    for nrhs in (1, 7):
        shp = (lambda n: (n,)) if nrhs == 1 else (lambda n: (n, nrhs))
        x1 = torch.from_numpy(rng.standard_normal(shp(2500))).cuda()
        x2 = torch.from_numpy(rng.standard_normal(shp(1800))).cuda()
        ys = matvec_batch([g1, g2], [x1, x2])
        for g, x, y in ((g1, x1, ys[0]), (g2, x2, ys[1])):
            assert torch.equal(y, g.matvec(x))
    g1.free()
    g2.free()
