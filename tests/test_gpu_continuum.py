"""GPU parity of continuum storage (the accessor remark of Sec. 4.3, reading
R11: per block the fewest fraction bits t in [7, 23] that the precision rule
allows, 9 + t bits per stored entry) against the oracle's
build(continuum=True), through the C ABI.

Bars: tree, partition, ranks and every block's t bit for bit (except decisions
inside the tie windows of parity_util); products (H and H^T, one and several
right-hand sides) within 1e-2 tol of the oracle's, within 10 tol of the dense
product; and within 1e-12 (relative) of the fp64 product of the GPU's own
exported factors, which checks the in-kernel decoding of the packed entries
(every width from 16 to 32 bits appears across the cases)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import format_window, rank_window, exported_product, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


ALIGNED = (7, 15, 23)        # continuum = 2: 16-, 24- and 32-bit entries


def _pair(P, kind, tol, eta, ell, leaf, normals=None, io="f64", mode=1):
    from paper_2604_09147_amd import HMatrix
    g = HMatrix(P, kind, tol, eta, ell, leaf, normals=normals, io_dtype=io, continuum=mode)
    o = O.build(P, O.Kernel(kind, normals=normals), tol, eta, ell, leaf, continuum=True,
                cont_ts=ALIGNED if mode == 2 else None)
    return g, o


def _compare(g, o):
    """Structure bit for bit; ranks and fraction bits outside tie windows."""
    bl = g.blocks()
    st = O.structure_arrays(o)
    assert np.array_equal(g.perm(), st["perm"])
    for key_g, key_o in (("level", "level"), ("box_i", "i"), ("box_j", "j"), ("kind", "kind")):
        assert np.array_equal(bl[key_g], st[key_o]), key_g
    assert np.array_equal(bl["lowrank"].astype(bool), st["lowrank"])
    t_o = np.array([sb.t if (sb.lowrank and sb.fmt == O.FMT_CONT) else 0 for sb in o.blocks])
    fmt_o = np.array([W.FMT_FP64 if not sb.lowrank else (4 if sb.fmt == O.FMT_CONT else sb.fmt)
                      for sb in o.blocks])
    ties = 0
    for q, sb in enumerate(o.blocks):
        same = (bl["rank"][q] == st["rank"][q] and bl["frac_bits"][q] == t_o[q] and
                bl["format"][q] == fmt_o[q])
        if same:
            continue
        c = sb.comp
        if bl["rank"][q] != st["rank"][q]:
            w = rank_window(min(sb.blk.m, sb.blk.n), c.sketch, o.eps)
            near = [math.isfinite(t) and abs(t - c.thr) <= w * c.thr for t in (c.tail, c.tail_prev)]
            assert any(near) and abs(int(bl["rank"][q]) - int(st["rank"][q])) == 1, q
        else:
            # the t decision: u_t^2 2^(d l) ||H~_b||^2 against eps^2 ||H~||^2,
            # at either of the two choices
            w = format_window(sb.rank, min(sb.blk.m, sb.blk.n), len(o.blocks))
            cand = {int(bl["frac_bits"][q]), int(t_o[q])} - {0}
            marg = [((2.0 ** -(u + 1)) ** 2 * 2.0 ** (o.d * sb.blk.level) * sb.nb2) /
                    (o.eps ** 2 * o.total2) for u in cand | {u - 1 for u in cand}]
            assert any(abs(m - 1.0) <= w for m in marg), (q, bl["frac_bits"][q], t_o[q], marg)
        ties += 1
    return bl, ties


def _products(g, o, P, kern, tol, nrhs=1, trans=False, dense=True, io="f64"):
    torch = _torch()
    rng = np.random.default_rng(nrhs + 7 * trans)
    shape = (P.shape[0],) if nrhs == 1 else (P.shape[0], nrhs)
    dt = torch.float32 if io == "f32" else torch.float64
    xd = torch.from_numpy(rng.standard_normal(shape)).to(dt).cuda()
    y = (g.matvec_t(xd) if trans else g.matvec(xd)).double().cpu().numpy()
    x = xd.double().cpu().numpy()
    yo = O.matvec_t(o, x) if trans else O.matvec(o, x)
    bar = max(1e-2 * tol, 2.0 ** -22) if io == "f32" else 1e-2 * tol
    assert rel(y, yo) <= bar, (rel(y, yo), bar)
    if io == "f64":
        ye, _ = exported_product(g, x, trans)
        assert rel(y, ye) <= 1e-12, rel(y, ye)
    if dense:
        yd = O.dense_matvec_t(P, kern, x) if trans else O.dense_matvec(P, kern, x)
        assert rel(y, yd) <= 10 * tol, rel(y, yd)


@pytest.mark.parametrize("tol,mode", [(1e-3, 1), (1e-6, 1), (1e-9, 1), (1e-4, 2), (1e-7, 2)])
def test_continuum_2d_log_against_the_oracle(tol, mode):
    rng = np.random.default_rng(70)
    P = rng.random((3000, 2))
    g, o = _pair(P, W.LOG, tol, 1.0, -1, 32, mode=mode)
    bl, ties = _compare(g, o)
    widths = set(9 + bl["frac_bits"][bl["format"] == 4])
    print(f"continuum 2D log tol {tol} mode {mode}: widths {sorted(widths)}, ties {ties}", flush=True)
    if mode == 2:
        assert widths <= {16, 24, 32}
    k = O.Kernel(W.LOG)
    for trans in (False, True):
        _products(g, o, P, k, tol, trans=trans)
        _products(g, o, P, k, tol, nrhs=3, trans=trans, dense=False)
    g.free()


def test_continuum_3d_laplace_recipe_and_derived_handle():
    # the benchmark recipe at N = 2^14 (L = 2): leaves of 256 points
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    p = W.cfg_3d_laplace(n=1 << 14, switch_level=-1)
    g = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                continuum=True)
    o = O.build(p.points, O.Kernel(p.kernel, scale=p.scale), p.tol, p.eta, p.switch_level,
                p.leaf_size, continuum=True)
    bl, _ = _compare(g, o)
    k = O.Kernel(p.kernel, scale=p.scale)
    _products(g, o, p.points, k, p.tol)
    _products(g, o, p.points, k, p.tol, trans=True)
    _products(g, o, p.points, k, p.tol, nrhs=16, dense=False)
    # continuum storage derived from an fp64 handle holds the same structure and
    # gives bit for bit the products of the direct build
    h64 = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                  uniform_fp64=True)
    hd = h64.derive(continuum=1)
    bd = hd.blocks()
    assert np.array_equal(bd["frac_bits"], bl["frac_bits"]) and np.array_equal(bd["rank"], bl["rank"])
    x = torch.randn(p.n, dtype=torch.float64, device="cuda")
    assert torch.equal(hd.matvec(x), g.matvec(x))
    s, s64 = hd.stats(), h64.stats()
    assert s["blocks_by_format"][4] > 0
    assert s["matvec_bytes"] < s64["matvec_bytes"]
    # the byte-aligned widths, derived, against the oracle's rule over t = 7, 15, 23
    ha = h64.derive(continuum=2)
    oa = O.build(p.points, O.Kernel(p.kernel, scale=p.scale), p.tol, p.eta, p.switch_level,
                 p.leaf_size, continuum=True, cont_ts=ALIGNED)
    _compare(ha, oa)
    _products(ha, oa, p.points, k, p.tol)
    _products(ha, oa, p.points, k, p.tol, trans=True, dense=False)
    _products(ha, oa, p.points, k, p.tol, nrhs=5, dense=False)
    for h in (g, hd, h64, ha):
        h.free()


def test_continuum_long_columns_and_f32_io():
    # 1D HODLR with level-1 columns of about 8200 rows (the inner-product
    # kernel's global-memory path) and fp32 inputs / outputs
    rng = np.random.default_rng(17)
    P = rng.random((16384, 1))
    tol = 1e-6
    g, o = _pair(P, W.INV_R, tol, 1.0, 0, 256, io="f32")
    _compare(g, o)
    k = O.Kernel(W.INV_R)
    _products(g, o, P, k, tol, io="f32")
    _products(g, o, P, k, tol, io="f32", trans=True)
    g.free()
