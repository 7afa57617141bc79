"""Shared helpers of the GPU parity tests: build the same problem with the HIP
library and with the oracle, compare structure (bit for bit, with the tie rule)
and products."""
from __future__ import annotations

import math

import numpy as np

import workloads as W
from oracle import hh_oracle as O

U64 = 2.0 ** -53

# The C header's codes of the formats that the oracle numbers differently
# (oracle: q43 = 4, continuum = 5; C: continuum = 4, q43 = 5).
HH_FMT_CONT, HH_FMT_Q43 = 4, 5
_GPU_CODE = {W.FMT_Q43: HH_FMT_Q43, O.FMT_CONT: HH_FMT_CONT}


def gpu_format_code(oracle_fmt: int) -> int:
    return _GPU_CODE.get(int(oracle_fmt), int(oracle_fmt))


def rank_window(pmin: int, sketch: int, eps: float) -> float:
    """Relative distance of a discarded tail from eps^2 ||H_b||^2 within which
    two correct fp64 implementations may decide the rank differently.

    The tail t_k = sum_{r > k} sigma_r^2 (plus ||H - Q Q^T H||^2 on the
    randomized path) is compared with thr = eps^2 ||H_b||_F^2 >= eps^2
    sigma_1^2. Singular values from two backward-stable SVDs (different
    algorithms and summation orders) differ by about c u sigma_1 with c ~
    sqrt(p), so |dt_k| <= 2 c u sigma_1 sum_{r > k} sigma_r + p u t_k <=
    2 c u sigma_1 sqrt(p t_k) + p u t_k, i.e. relative to thr at most
    2 p u / eps + p u. The residual of the randomized path, an explicit
    difference H - Q B whose entries carry errors of about (s + 2) u |H_ij|,
    adds 4 (s + 2) u / eps."""
    p = max(int(pmin), 1)
    s = max(int(sketch), 0)
    return (2.0 * p + (4.0 * (s + 2) if s > 0 else 0.0)) * U64 / eps + p * U64


def format_window(rank: int, pmin: int, n_blocks: int) -> float:
    """Relative width of a format tie: ||H~_b||^2 = sum_{r <= k} sigma_r^2 differs
    between implementations by about (2 sqrt(p) + k) u relative, ||H~||^2 (a sum
    over every block in another order) by about n_blocks u."""
    return (2.0 * max(pmin, 1) ** 0.5 + rank + n_blocks + 8.0) * U64


def build_pair(points, kernel, tol, eta, ell, leaf, mask=0xF, uniform=False, normals=None,
               scale=1.0, h=1.0, io="f64", seed=0):
    from paper_2604_09147_amd import HMatrix
    g = HMatrix(points, kernel, tol, eta, ell, leaf, scale=scale, h=h, normals=normals, mask=mask,
                uniform_fp64=uniform, io_dtype=io, seed=seed)
    k = O.Kernel(kernel, scale=scale, h=h, normals=normals)
    o = O.build(points, k, tol, eta, ell, leaf, mask=mask, uniform=uniform, seed=seed)
    return g, o


def rank_tie(sb, eps) -> bool:
    c = sb.comp
    if c is None:
        return False
    w = rank_window(min(sb.blk.m, sb.blk.n), c.sketch, eps)
    near = lambda t: math.isfinite(t) and abs(t - c.thr) <= w * c.thr
    return near(c.tail) or near(c.tail_prev)


def format_tie(hm, sb) -> bool:
    if not sb.lowrank or hm.uniform:
        return False
    w = format_window(sb.rank, min(sb.blk.m, sb.blk.n), len(hm.blocks))
    for f in (W.FMT_Q43, W.FMT_BF16, W.FMT_FP16, W.FMT_FP32):
        if hm.mask & (1 << f):
            r = O.format_margin(sb.nb2, hm.total2, sb.blk.level, hm.d, hm.eps, f)
            if abs(r - 1.0) <= w:
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
        f_ok = bl["format"][q] == gpu_format_code(st["fmt"][q])
        if r_ok and f_ok:
            continue
        if (not r_ok and rank_tie(sb, o.eps) and abs(int(bl["rank"][q]) - int(st["rank"][q])) == 1) or \
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
    lane sums of about P/64 terms in fp32; q43 blocks likewise), so per such block
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
            if bl["format"][q] in (W.FMT_FP16, W.FMT_BF16, HH_FMT_Q43):
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
