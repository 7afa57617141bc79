"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function include/hh.h declares, the host planner (tree + partition)
matches the oracle bit for bit, the storage rounding matches the oracle's, and
invalid arguments are rejected before any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_2604_09147_amd import hh
    if not os.path.exists(hh.LIB_PATH):
        pytest.skip("native library not built")
    return hh


def test_library_exports_every_declared_function():
    hh = _lib_or_skip()
    header = open(os.path.join(ROOT, "include", "hh.h")).read()
    declared = set(re.findall(r"\b(hh_[a-z_]+)\s*\(", header))
    assert declared == set(hh.EXPORTS)
    lib = hh.lib()
    for name in declared:
        assert hasattr(lib, name), name


def _compare_plan(points, eta, ell, leaf):
    hh = _lib_or_skip()
    pl = hh.plan(points, eta, ell, leaf)
    t = O.build_tree(points, leaf)
    bl = O.partition(t, eta, ell)
    assert pl["L"] == t.L and pl["ell"] == O.resolve_switch_level(ell, t.L)
    assert np.array_equal(pl["perm"], t.perm)
    assert len(bl) == pl["level"].size
    want = np.array([(b.level, b.i, b.j, b.kind, b.ib, b.ie, b.jb, b.je) for b in bl], dtype=np.int64)
    got = np.stack([pl[k].astype(np.int64) for k in
                    ("level", "i", "j", "kind", "ib", "ie", "jb", "je")], axis=1)
    assert np.array_equal(want, got)


@pytest.mark.parametrize("n,d,leaf,eta,ell,seed", [
    (1, 2, 8, 1.0, -1, 0), (7, 3, 8, 1.0, -1, 1), (300, 1, 8, 1.0, 2, 2),
    (4096, 2, 64, 1.0, 2, 101), (3001, 2, 32, math.sqrt(2), -1, 3), (3001, 2, 32, 1.0, 0, 4),
    (3001, 2, 32, 0.7, 4, 5), (5000, 3, 16, 1.5, 2, 6), (5000, 3, 16, math.sqrt(3), 3, 7),
    (5000, 3, 16, 2.5, 0, 8)])
def test_plan_matches_oracle(n, d, leaf, eta, ell, seed):
    rng = np.random.default_rng(seed)
    P = rng.random((n, d))
    _compare_plan(P, eta, ell, leaf)


def test_plan_matches_oracle_clustered_points():
    rng = np.random.default_rng(9)
    P = np.concatenate([rng.random((2000, 2)) * 0.01, rng.random((500, 2)), [[5.0, 5.0]]])
    _compare_plan(P, 1.0, 2, 16)
    _compare_plan(np.repeat(rng.random((40, 3)), 5, axis=0), 1.5, -1, 8)   # coincident points


def test_plan_full_size_headline_structure():
    # 3D Laplace workload: N = 2^20, leaf 256 (L = 4), eta 1.5, switch 3
    p = W.cfg_3d_laplace()
    _compare_plan(p.points, p.eta, p.switch_level, p.leaf_size)


def test_plan_full_size_2d_and_double_layer():
    p = W.cfg_2d_inv_r()
    _compare_plan(p.points, p.eta, p.switch_level, p.leaf_size)
    q = W.cfg_double_layer()
    _compare_plan(q.points, q.eta, q.switch_level, q.leaf_size)


def test_quantize_matches_oracle_rounding():
    hh = _lib_or_skip()
    rng = np.random.default_rng(3)
    v = rng.standard_normal(20000) * 10.0 ** rng.integers(-12, 8, 20000)
    # exact midpoints of fp16 / bf16 neighbours, subnormal range and overflow
    g16 = np.arange(0, 0x7C00, 7, dtype=np.uint16).view(np.float16).astype(np.float64)
    v = np.concatenate([v, (g16[1:] + g16[:-1]) / 2, [2.0 ** -20, 3 * 2.0 ** -25, 65520.0, 1e300]])
    for fmt in (W.FMT_FP64, W.FMT_FP32, W.FMT_FP16, W.FMT_BF16):
        for e in (0, -3, 7):
            ref = np.ldexp(O.round_to(np.ldexp(v, -e), fmt), e)
            got = hh.quantize(v, fmt, e)
            same = (got == ref) | (np.isnan(got) & np.isnan(ref))
            assert same.all(), (fmt, e, v[~same][:5], got[~same][:5], ref[~same][:5])


def test_quantize_q43_matches_oracle_rounding():
    # q43 (C code 5, oracle code 4): every code's midpoints with its neighbours,
    # the subnormal range, random magnitudes; past 240 the library saturates
    # where the oracle returns inf (stored factors are scaled to [64, 128))
    hh = _lib_or_skip()
    codes = np.arange(0, 0x78, dtype=np.uint8)
    vals = np.ldexp(np.where(codes >> 3 > 0, 8.0 + (codes & 7), (codes & 7).astype(np.float64)),
                    np.maximum(codes.astype(np.int64) >> 3, 1) - 10)
    assert np.array_equal(O.round_q43(vals), vals)
    mids = (vals[1:] + vals[:-1]) / 2
    rng = np.random.default_rng(8)
    v = rng.standard_normal(20000) * 2.0 ** rng.uniform(-14, 9, 20000)
    v = np.concatenate([v, vals, -vals, mids, -mids, np.nextafter(mids, 0), np.nextafter(mids, 1e9),
                        [2.0 ** -10, 3 * 2.0 ** -11, 2.0 ** -11, 247.9, 248.0, 1e6]])
    for e in (0, -3, 7):
        ref = np.ldexp(O.round_q43(np.ldexp(v, -e)), e)
        ref = np.where(np.isinf(ref), np.sign(ref) * np.ldexp(240.0, e), ref)
        got = hh.quantize(v, hh.FMT_Q43, e)
        same = got == ref
        assert same.all(), (e, v[~same][:5], got[~same][:5], ref[~same][:5])
    with pytest.raises(hh.HHError):
        hh.quantize(v[:4], hh.FMT_CONT, 0)


def test_q43_code_read_as_fp16_is_the_value_times_2_to_the_minus_8():
    # the product kernels widen a q43 code by moving its sign to bit 15 and its
    # exponent and fraction to bits 7..14 of an fp16; that is exact for every
    # code (subnormals included) once the block's scale carries 2^8 per factor
    codes = np.arange(256, dtype=np.uint16)
    h16 = (((codes & 0x7F) << 7) | ((codes & 0x80) << 8)).astype(np.uint16).view(np.float16)
    e, f = (codes >> 3) & 15, codes & 7
    val = np.ldexp(np.where(e > 0, 8.0 + f, f.astype(np.float64)), np.maximum(e.astype(np.int64), 1) - 10)
    val = np.where(codes & 0x80, -val, val)
    assert np.array_equal(h16.astype(np.float64) * 256.0, val)
    finite = codes[(codes & 0x7F) <= 0x77]
    assert np.array_equal(O.round_q43(val[finite]), val[finite])


def test_invalid_arguments_rejected_on_host():
    hh = _lib_or_skip()
    P = np.random.default_rng(0).random((100, 2))
    cases = [dict(points=P[:0], eta=1.0, switch_level=-1, leaf_size=8),
             dict(points=np.zeros((10, 4)), eta=1.0, switch_level=-1, leaf_size=8),
             dict(points=P, eta=0.0, switch_level=-1, leaf_size=8),
             dict(points=P, eta=1.0, switch_level=9, leaf_size=8),
             dict(points=P, eta=1.0, switch_level=-2, leaf_size=8),
             dict(points=P, eta=1.0, switch_level=-1, leaf_size=0),
             dict(points=np.where(P > 0.5, np.nan, P), eta=1.0, switch_level=-1, leaf_size=8)]
    for kw in cases:
        with pytest.raises(hh.HHError) as ei:
            hh.plan(**kw)
        assert ei.value.status == hh.HH_EINVAL
    # hh_build validates before touching the device
    lib = hh.lib()
    out = C.c_void_p()
    pts = np.ascontiguousarray(P)
    k = hh.Kernel(hh.INV_R, 1.0, 1.0, None)
    for tol, kern in ((0.0, k), (1.5, k), (1e-6, hh.Kernel(99, 1.0, 1.0, None)),
                      (1e-6, hh.Kernel(hh.DOUBLE_LAYER, 1.0, 1.0, None))):
        st = lib.hh_build(pts.ctypes.data_as(C.POINTER(C.c_double)), 100, 2, C.byref(kern), tol,
                          1.0, -1, 8, None, C.byref(out))
        assert st == hh.HH_EINVAL and not out.value
        assert lib.hh_last_error()
    # mask bit 4 is the continuum code, not a format the rule picks
    opt = hh.Options(precision_mask=0x1F)
    st = lib.hh_build(pts.ctypes.data_as(C.POINTER(C.c_double)), 100, 2, C.byref(k), 1e-6, 1.0, -1,
                      8, C.byref(opt), C.byref(out))
    assert st == hh.HH_EINVAL and not out.value and b"0x2F" in lib.hh_last_error()
    assert lib.hh_matvec(None, None, None, 1, None) == hh.HH_EINVAL
    lib.hh_free(None)


def test_switch_level_search_rejects_bad_arguments_on_host():
    # argument errors come back before any build touches the device
    hh = _lib_or_skip()
    lib = hh.lib()
    P = np.ascontiguousarray(np.random.default_rng(1).random((2048, 2)))   # L = 3 at leaf 32
    pp = P.ctypes.data_as(C.POINTER(C.c_double))
    k = hh.Kernel(hh.INV_R, 1.0, 1.0, None)
    lvl = C.c_int32(7)
    s = np.zeros(8)
    sp = s.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.hh_switch_level_search(pp, 2048, 2, C.byref(k), 1e-6, 1.0, 32, None, None, sp, sp,
                                      8) == hh.HH_EINVAL
    # s1 / s2 need L + 1 = 4 entries
    assert lib.hh_switch_level_search(pp, 2048, 2, C.byref(k), 1e-6, 1.0, 32, None, C.byref(lvl),
                                      sp, None, 3) == hh.HH_EINVAL
    assert lvl.value == -1 and "L + 1" in lib.hh_last_error().decode()
    for tol, eta, leaf in ((0.0, 1.0, 32), (1e-6, 0.0, 32), (1e-6, 1.0, 0)):
        assert lib.hh_switch_level_search(pp, 2048, 2, C.byref(k), tol, eta, leaf, None,
                                          C.byref(lvl), None, None, 0) == hh.HH_EINVAL


@pytest.mark.parametrize("t", [7, 10, 15, 16, 17, 22, 23])
def test_continuum_rounding_matches_oracle(t):
    # the library's continuum rounding (f64_to_cont_rne, host side) against the
    # oracle's round_fp, written independently: random magnitudes over the whole
    # exponent range, exact ties between neighbours, the gradual-underflow range
    # and the overflow edge; t = 7 and t = 23 also against bf16 / fp32 rounding
    hh = _lib_or_skip()
    rng = np.random.default_rng(t)
    xs = [rng.standard_normal(4000) * 10.0 ** rng.uniform(-44, 38, 4000)]
    k = rng.integers(1 << t, 1 << (t + 1), 2000)
    e = rng.integers(-125, 127, 2000)
    xs.append(np.ldexp(2.0 * k + 1.0, e - t - 1) * rng.choice([-1.0, 1.0], 2000))   # ties
    ks = rng.integers(0, 1 << t, 1000)
    xs.append(np.ldexp(2.0 * ks + 1.0, -126 - t - 1))                                  # subnormal ties
    xs.append(rng.uniform(0.0, 2.0 ** -126, 1000))
    top = (2.0 - 2.0 ** -t) * 2.0 ** 127
    xs.append(np.array([top, top * (1 + 2.0 ** -(t + 2)), top * (1 + 2.0 ** -(t + 1)), 2.0 ** 128,
                        -top, 0.0, -0.0, 2.0 ** -150, 2.0 ** -149, 3.0 * 2.0 ** -151]))
    x = np.concatenate(xs)
    got = hh.quantize_cont(x, t)
    want = O.round_fp(x, t)
    bad = np.flatnonzero(~((got == want) | (np.isnan(got) & np.isnan(want))))
    assert bad.size == 0, (x[bad[:5]], got[bad[:5]], want[bad[:5]])
    assert np.array_equal(np.signbit(got[x == 0.0]), np.signbit(x[x == 0.0]))
    if t == 23:
        with np.errstate(over="ignore"):
            assert np.array_equal(got, x.astype(np.float32).astype(np.float64))
    if t == 7:
        assert np.array_equal(got, O.round_bf16(x))
