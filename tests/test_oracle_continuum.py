"""Pins of the oracle's continuum storage (Sec. 4.3 accessor remark; the
format is a reading: 8-bit exponent, t fraction bits, ties to even).

* t = 23 is IEEE single (numpy's own cast, subnormals and exact ties
  included), t = 10 is IEEE half inside half's normal range, t = 7 is the
  oracle's bf16 (itself pinned by brute force);
* any t: the nearest multiple of the binade's spacing with ties to the even
  multiple, computed in exact rational arithmetic;
* the relative error stays below u = 2^-(t+1) and reaches u / (1 + u) at the
  first tie;
* the rule takes the smallest passing t (ties pass) and never asks for more
  bits than the fixed-format rule's choice;
* built matrices keep eq:need_mvp per block and Thm amp_throrem globally, and
  store fewer bits than the fixed formats {fp64, fp32, bf16}."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O


def test_t23_is_ieee_single_and_t10_is_ieee_half():
    rng = np.random.default_rng(23)
    x = rng.standard_normal(4000) * 2.0 ** rng.integers(-150, 120, 4000)
    f32 = np.float32
    # exact ties between neighbouring singles, normal and subnormal
    a = rng.standard_normal(300).astype(f32) * f32(2.0) ** rng.integers(-140, 100, 300).astype(f32)
    b = np.nextafter(a, f32(np.inf))
    ties = (a.astype(np.float64) + b.astype(np.float64)) / 2.0
    for v in (x, ties):
        ok = np.abs(v) < float(np.finfo(f32).max)
        assert np.array_equal(O.round_fp(v[ok], 23), v[ok].astype(f32).astype(np.float64))
    h = rng.uniform(-1, 1, 4000) * 2.0 ** rng.integers(-14, 15, 4000)
    h = h[(np.abs(h) >= 2.0 ** -14) & (np.abs(h) <= 65504.0)]
    assert np.array_equal(O.round_fp(h, 10), h.astype(np.float16).astype(np.float64))


def test_t7_is_bf16():
    rng = np.random.default_rng(7)
    x = rng.standard_normal(4000) * 10.0 ** rng.integers(-40, 38, 4000)
    assert np.array_equal(O.round_fp(x, 7), O.round_bf16(x))


@pytest.mark.parametrize("t", [8, 12, 15, 16, 18, 21])
def test_any_t_is_the_nearest_even_multiple_exactly(t):
    rng = np.random.default_rng(t)
    x = rng.standard_normal(300) * 2.0 ** rng.integers(-130, 100, 300)
    got = O.round_fp(x, t)
    for xi, gi in zip(x, got):
        e = max(math.frexp(abs(xi))[1] - 1, -126)
        ulp = Fraction(2) ** (e - t)
        k = round(Fraction(abs(xi)) / ulp)           # Python rounds a Fraction half to even
        want = math.copysign(float(k * ulp), xi)
        assert gi == want, (t, xi, gi, want)
    # the first tie above 1 rounds down to 1 (even multiple)
    assert O.round_fp(np.array([1.0 + 2.0 ** -(t + 1)]), t)[0] == 1.0


@pytest.mark.parametrize("t", [7, 11, 16, 19, 23])
def test_relative_error_below_unit_roundoff(t):
    rng = np.random.default_rng(100 + t)
    x = 2.0 ** rng.uniform(-100, 100, 100000)
    rel = np.abs(O.round_fp(x, t) - x) / x
    u = 2.0 ** -(t + 1)
    assert rel.max() <= u
    tie = 1.0 + u
    assert (tie - O.round_fp(np.array([tie]), t)[0]) / tie == pytest.approx(u / (1 + u), rel=1e-12)


def test_rule_takes_the_smallest_passing_t():
    d, level, eps, total2 = 3, 3, 1e-6, 1.0
    for t in range(7, 24):
        u = 2.0 ** -(t + 1)
        tie = (eps * eps) / ((u * u) * 2.0 ** (d * level))   # exact tie for this t
        assert O.choose_fraction_bits(tie, total2, level, d, eps) == t
        assert O.choose_fraction_bits(tie * (1 + 2 ** -40), total2, level, d, eps) == (t + 1 if t < 23 else None)
    # never more precision than the fixed-format rule asks for
    rng = np.random.default_rng(5)
    for _ in range(2000):
        nb2 = 10.0 ** rng.uniform(-30, 0)
        lvl = int(rng.integers(1, 5))
        fmt = O.choose_format(nb2, total2, lvl, d, eps, 0xF)
        t = O.choose_fraction_bits(nb2, total2, lvl, d, eps)
        if fmt == W.FMT_FP64:
            assert t is None
        else:
            assert t is not None and 2.0 ** -(t + 1) >= O.UNIT[fmt]


@pytest.mark.parametrize("eps", [1e-6, 1e-3])
def test_continuum_build_keeps_the_bounds_and_saves_bits(eps):
    rng = np.random.default_rng(21)
    P = rng.random((1500, 2))
    k = O.Kernel(W.LOG)
    hc = O.build(P, k, eps, 1.0, -1, 32, continuum=True)
    used = {sb.t for sb in hc.blocks if sb.lowrank and sb.fmt == O.FMT_CONT}
    assert len(used) > 1                            # several widths in one matrix
    for sb in hc.blocks:
        if sb.lowrank and sb.rank:
            u = O.block_unit(sb)
            dlt = np.linalg.norm(sb.Ut @ sb.Vt.T - sb.U @ sb.V.T)
            assert dlt <= (2 + math.sqrt(sb.rank) * u) * u * math.sqrt(sb.nb2) * (1 + 1e-9)
    H = O.dense_matrix(P, k)
    A, cover = O.assemble(hc, "stored")
    assert cover.min() == 1 and cover.max() == 1
    assert np.linalg.norm(H - A) <= O.global_bound(hc.d, hc.eta, hc.tree.L, hc.ell) * eps * np.linalg.norm(H)
    x = rng.standard_normal(1500)
    assert np.allclose(O.matvec(hc, x), A @ x, rtol=1e-12, atol=1e-12 * np.abs(A @ x).max())
    hf = O.build(P, k, eps, 1.0, -1, 32, mask=0xB)  # fp64, fp32, bf16
    assert O.storage(hc)["lowrank"] < O.storage(hf)["lowrank"]
