"""Shared helpers of the GPU parity tests: build the same problem with the HIP
library and with the oracle, compare structure (bit for bit, with the tie rule)
and products."""
from __future__ import annotations

import math

import numpy as np

import workloads as W
from oracle import hh_oracle as O

TIE_REL = 1e-6      # rank / format decisions this close to their threshold are ties


def build_pair(points, kernel, tol, eta, ell, leaf, mask=0xF, uniform=False, normals=None,
               scale=1.0, h=1.0, io="f64", seed=0):
    from paper_2604_09147_amd import HMatrix
    g = HMatrix(points, kernel, tol, eta, ell, leaf, scale=scale, h=h, normals=normals, mask=mask,
                uniform_fp64=uniform, io_dtype=io, seed=seed)
    k = O.Kernel(kernel, scale=scale, h=h, normals=normals)
    o = O.build(points, k, tol, eta, ell, leaf, mask=mask, uniform=uniform, seed=seed)
    return g, o


def rank_tie(sb) -> bool:
    c = sb.comp
    if c is None:
        return False
    near = lambda t: math.isfinite(t) and abs(t - c.thr) <= TIE_REL * c.thr
    return near(c.tail) or near(c.tail_prev)


def format_tie(hm, sb) -> bool:
    if not sb.lowrank or hm.uniform:
        return False
    for f in (W.FMT_BF16, W.FMT_FP16, W.FMT_FP32):
        if hm.mask & (1 << f):
            r = O.format_margin(sb.nb2, hm.total2, sb.blk.level, hm.d, hm.eps, f)
            if abs(r - 1.0) <= 1e-9:
                return True
    return False


def compare_structure(g, o) -> list:
    """Assert the GPU structure equals the oracle's; return indices of tie blocks
    whose rank or format differ (allowed)."""
    bl = g.blocks()
    st = O.structure_arrays(o)
    assert np.array_equal(g.perm(), st["perm"])
    for key_g, key_o in (("level", "level"), ("box_i", "i"), ("box_j", "j")):
        assert np.array_equal(bl[key_g], st[key_o]), key_g
    assert np.array_equal(bl["lowrank"].astype(bool), st["lowrank"])
    assert np.array_equal(bl["kind"], st["kind"])
    ties = []
    for q, sb in enumerate(o.blocks):
        r_ok = bl["rank"][q] == st["rank"][q]
        f_ok = bl["format"][q] == st["fmt"][q]
        if r_ok and f_ok:
            continue
        if (not r_ok and rank_tie(sb) and abs(int(bl["rank"][q]) - int(st["rank"][q])) == 1) or \
           (r_ok and not f_ok and format_tie(o, sb)):
            ties.append(q)
            continue
        raise AssertionError(f"block {q}: rank {bl['rank'][q]} vs {st['rank'][q]}, "
                             f"format {bl['format'][q]} vs {st['fmt'][q]}")
    return ties


def exported_product(g, x, trans=False):
    """fp64 product with the GPU's own stored factors (exported and decoded),
    plus an elementwise bound on the kernel's deviation from it: fp16 / bf16
    blocks form their inner products in fp32 (x rounded to fp32, products and
    lane sums of about P/64 terms in fp32), so per such block
    |err| <= gamma_P |A| (|B|^T |x|) with gamma_P = (P/64 + 4) 2^-24."""
    perm = g.perm()
    n = g.n
    x2 = np.asarray(x, dtype=np.float64).reshape(n, -1)
    xt = x2[perm]
    yt = np.zeros_like(xt)
    bt = np.zeros_like(xt)
    bl = g.blocks()
    for q in range(bl["level"].size):
        ib, ie, jb, je = (int(bl[k][q]) for k in ("row_begin", "row_end", "col_begin", "col_end"))
        A, B = g.block_factors(q)
        if bl["lowrank"][q]:
            if bl["rank"][q] == 0:
                continue
            if trans:
                A, B, ib, ie, jb, je = B, A, jb, je, ib, ie
            yt[ib:ie] += A @ (B.T @ xt[jb:je])
            if bl["format"][q] in (W.FMT_FP16, W.FMT_BF16):
                P = 4 * (-(-(je - jb) // 4)) + 64          # padded length, generous
                gam = (P / 64.0 + 4.0) * 2.0 ** -24
                bt[ib:ie] += gam * (np.abs(A) @ (np.abs(B).T @ np.abs(xt[jb:je])))
        else:
            if trans:
                yt[jb:je] += A.T @ xt[ib:ie]
            else:
                yt[ib:ie] += A @ xt[jb:je]
    y = np.empty_like(yt)
    y[perm] = yt
    b = np.empty_like(bt)
    b[perm] = bt
    return y.reshape(np.shape(x)), b.reshape(np.shape(x))


def within_kernel_bound(y, ye, bound, slack=1e-12) -> bool:
    return bool(np.all(np.abs(y - ye) <= bound + slack * np.max(np.abs(ye))))


def rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))
