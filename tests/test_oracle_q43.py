"""Pins of the oracle's 8-bit quarter precision q43 (the paper's format table:
1 sign, 4 exponent, 3 fraction bits, x_min = 1.56e-2, x_max = 2.4e2, exponents
-6..7) and of its use as the lowest precision of the adaptive rule.

* the code table decoded from the format's definition (written here, not in
  the oracle) has the table's x_min, x_max and exponent range;
* rounding is the nearest table value, ties to the even code, by brute force,
  with overflow to inf from 248 (halfway to the next binade) on;
* codes round-trip; the relative rounding error over the normal range stays
  below 2^-4 and reaches 2^-4 / (1 + 2^-4) at the first tie;
* the per-factor scale puts the largest entry in [64, 128);
* the precision rule picks q43 exactly when u = 2^-4 passes (ties pass) and
  only when its mask bit is set;
* the paper's setting with q43 available (log r in [-1,1]^2, N = 6400, L = 4,
  ell = 3, eps = 1e-2): some blocks are stored in q43, every block keeps
  eq:need_mvp and the whole matrix the bound of Thm amp_throrem."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O


def _decode(code: int) -> float:
    s = -1.0 if code & 0x80 else 1.0
    field = (code >> 3) & 0xF
    frac = code & 0x7
    if field == 0xF:
        return math.nan                            # reserved (inf / nan)
    if field == 0:
        return s * frac * 2.0 ** -9                # subnormal: 0.fff x 2^-6
    return s * (1.0 + frac / 8.0) * 2.0 ** (field - 7)


def _table():
    vals = {c: _decode(c) for c in range(256)}
    return {c: v for c, v in vals.items() if not math.isnan(v)}


def test_code_table_matches_the_format_table():
    t = _table()
    pos = sorted({v for v in t.values() if v > 0})
    normals = [v for v in pos if v >= 2.0 ** -6]
    assert len(t) == 240                          # 2 signs x 15 exponent fields x 8 fractions
    assert max(pos) == 240.0                      # printed x_max 2.4e2
    assert min(normals) == 2.0 ** -6              # printed x_min 1.56e-2
    assert abs(min(normals) - 1.56e-2) < 5e-5
    assert math.floor(math.log2(max(pos))) == 7 and math.floor(math.log2(min(normals))) == -6
    assert min(pos) == 2.0 ** -9                  # gradual underflow


def test_rounding_is_nearest_even_by_brute_force():
    t = _table()
    grid = np.array(sorted(set(t.values())))
    code_of = {}
    for c, v in t.items():
        if v != 0.0 or c == 0:
            code_of.setdefault(v, c)
    rng = np.random.default_rng(43)
    xs = list(rng.standard_normal(500) * 2.0 ** rng.integers(-12, 8, 500))
    mids = (grid[1:] + grid[:-1]) / 2.0            # exact ties
    xs += list(rng.choice(mids, 300))
    # beyond the grid (from 248 on) rounding overflows; checked below
    for x in (x for x in xs if abs(x) < 248.0):
        i = np.searchsorted(grid, x)
        lo, hi = grid[max(i - 1, 0)], grid[min(i, grid.size - 1)]
        if abs(x - lo) < abs(hi - x):
            want = lo
        elif abs(hi - x) < abs(x - lo):
            want = hi
        else:
            want = lo if code_of[lo] % 2 == 0 else hi
        got = float(O.round_q43(np.array([x]))[0])
        assert got == want, (x, got, want)
    # overflow: 247.99 stays at the largest value, 248 and beyond go to inf
    r = O.round_q43(np.array([247.99, 248.0, -300.0, 1e9]))
    assert r[0] == 240.0 and np.isposinf(r[1]) and np.isneginf(r[2]) and np.isposinf(r[3])


def test_codes_round_trip_and_unit_roundoff():
    t = _table()
    for c, v in t.items():
        if c == 0x80:                              # -0 encodes as 0x80 as well
            continue
        assert int(O.q43_bits(np.array([v]))[0]) == c, (c, v)
        assert float(O.round_q43(np.array([v]))[0]) == v
    rng = np.random.default_rng(4)
    x = 2.0 ** rng.uniform(-6, math.log2(240.0), 200000)
    rel = np.abs(O.round_q43(x) - x) / x
    assert rel.max() <= O.UNIT[W.FMT_Q43] == 2.0 ** -4
    tie = 1.0 + 2.0 ** -4                          # halfway between 1 and 1.125
    assert O.round_q43(np.array([tie]))[0] == 1.0
    assert (tie - 1.0) / tie == pytest.approx(2.0 ** -4 / (1 + 2.0 ** -4), rel=1e-15)


def test_scaling_puts_max_in_64_to_128():
    rng = np.random.default_rng(9)
    for mag in (1e-30, 1e-3, 1.0, 7e4, 1e20):
        F = rng.standard_normal((30, 4)) * mag
        stored, raw, e = O.quantize(F, W.FMT_Q43)
        mx = np.max(np.abs(np.ldexp(F, -e)))
        assert 64.0 <= mx < 128.0
        assert raw.dtype == np.uint8
        assert np.array_equal(stored, O.round_q43(np.ldexp(F, -e)))
        assert np.all(np.isfinite(stored))


def test_precision_rule_with_q43():
    d, level, eps, total2 = 2, 3, 1e-2, 1.0
    # u^2 2^(dl) nb2 <= eps^2 total2 with u = 2^-4: an exact tie passes
    nb2_tie = (eps * eps) / ((2.0 ** -8) * 2.0 ** (d * level))
    mask = 0x1F
    assert O.choose_format(nb2_tie, total2, level, d, eps, mask) == W.FMT_Q43
    assert O.choose_format(nb2_tie * (1 + 2 ** -40), total2, level, d, eps, mask) == W.FMT_BF16
    assert O.choose_format(nb2_tie / 4, total2, level, d, eps, 0xF) == W.FMT_BF16
    assert O.format_margin(nb2_tie, total2, level, d, eps, W.FMT_Q43) == 1.0


def test_paper_setting_with_q43_keeps_the_bounds():
    rng = np.random.default_rng(6400)
    P = rng.uniform(-1.0, 1.0, (6400, 2))
    k = O.Kernel(W.LOG)
    eps = 1e-2
    hm = O.build(P, k, eps, math.sqrt(2.0), -1, 25, mask=0x1F)
    assert hm.tree.L == 4 and hm.ell == 3
    fm = O.storage(hm)["blocks_by_format"]
    assert fm[W.FMT_Q43] > 0
    for sb in hm.blocks:
        if sb.lowrank and sb.rank:
            u = O.UNIT[sb.fmt]
            dlt = np.linalg.norm(sb.Ut @ sb.Vt.T - sb.U @ sb.V.T)
            assert dlt <= (2 + math.sqrt(sb.rank) * u) * u * math.sqrt(sb.nb2) * (1 + 1e-9)
    H = O.dense_matrix(P, k)
    A, cover = O.assemble(hm, "stored")
    assert cover.min() == 1 and cover.max() == 1
    c = O.global_bound(hm.d, hm.eta, hm.tree.L, hm.ell)
    assert np.linalg.norm(H - A) <= c * eps * np.linalg.norm(H)
    # q43 halves the bits of the bf16 blocks it replaces
    hm16 = O.build(P, k, eps, math.sqrt(2.0), -1, 25, mask=0xF)
    assert O.storage(hm)["lowrank"] < O.storage(hm16)["lowrank"]
