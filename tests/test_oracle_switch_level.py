"""Pins of the oracle's switching-level choice (Sec. 3.3: eq:S1, eq:S2, Alg. 2).

* the walk's stop rule on given gain sequences (strict growth continues, a tie
  or a loss stops, S2 asked for only where the walk reaches);
* S1(ell) - S2(ell) equals the difference of the total storage of two
  independent builds, H_s and H_h(ell), once their shared blocks (coarse
  interaction lists and diagonal) are checked to coincide;
* S1(L), the dense leaf neighbours of H_s, equals a brute-force count of the
  matrix entries whose leaf boxes are distinct and inadmissible;
* the walk's result against the brute-force arg max over every level;
* the paper's observation (Table tab:s1_s_2) that H_h needs less storage than
  H_s at ell = L - 1 for 1/r in 3D, with a ratio S1/S2 that falls as eps
  decreases (statistical: a smaller instance of the same recipe)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O


def _walk(L, s1, s2_values):
    asked = []

    def s2_fn(ell):
        asked.append(ell)
        return s2_values[ell]
    ell, gains = O.switch_level_search(L, np.asarray(s1, dtype=float), s2_fn)
    return ell, gains, asked


def test_stop_rule_on_given_gains():
    # gains S1 - S2 per level, L = 5
    s1 = [10.0] * 6
    # growing all the way down: ell* = 0, every level asked once
    ell, gains, asked = _walk(5, s1, {4: 9, 3: 8, 2: 7, 1: 6, 0: 5})
    assert ell == 0 and asked == [4, 3, 2, 1, 0] and gains[0] == 5.0
    # a peak at 3: the walk stops at the first loss and never asks below 2
    ell, gains, asked = _walk(5, s1, {4: 8, 3: 7, 2: 9, 1: 0, 0: 0})
    assert ell == 3 and asked == [4, 3, 2]
    # a tie stops the walk even if a deeper level would gain more
    ell, gains, asked = _walk(5, s1, {4: 10, 3: 0, 2: 0, 1: 0, 0: 0})
    assert ell == 5 and asked == [4]
    # a loss at L - 1 keeps H_s
    ell, gains, asked = _walk(5, s1, {4: 11, 3: 0, 2: 0, 1: 0, 0: 0})
    assert ell == 5 and gains == {5: 0.0, 4: -1.0}
    # L = 0: nothing to walk
    ell, gains, asked = _walk(0, [3.0], {})
    assert ell == 0 and asked == []


def _case_2d(seed=7):
    rng = np.random.default_rng(seed)
    return rng.random((2048, 2)), O.Kernel(W.INV_R), 1.0, 32


def _shared(hm, ell):
    """(level, i, j, rank, fmt) of the blocks H_s and H_h(ell) share."""
    out = []
    for sb in hm.blocks:
        b = sb.blk
        if b.kind == O.T_DIAG or (b.kind == O.T_FAR and b.level <= ell):
            out.append((b.level, b.i, b.j, sb.rank if sb.lowrank else -1, sb.fmt if sb.lowrank else -1))
    return out


@pytest.mark.parametrize("uniform", [True, False])
def test_s1_minus_s2_is_the_storage_difference(uniform):
    P, k, eta, leaf = _case_2d()
    eps = 1e-6
    L = O.build_tree(P, leaf).L
    hs = O.build(P, k, eps, eta, L, leaf, uniform=uniform)
    s1 = O.s1_by_level(hs)
    total_s = O.storage(hs)["total"]
    # S1(ell) - S1(ell + 1) is the interaction list of level ell + 1
    for ell in range(L):
        lvl = sum(O.block_words(sb) for sb in hs.blocks if sb.blk.kind == O.T_FAR and sb.blk.level == ell + 1)
        assert math.isclose(s1[ell] - s1[ell + 1], lvl, rel_tol=1e-12, abs_tol=1e-9)
    for ell in range(L):
        hh = O.build(P, k, eps, eta, ell, leaf, uniform=uniform)
        assert _shared(hh, ell) == _shared(hs, ell), ell
        gain = total_s - O.storage(hh)["total"]
        assert math.isclose(s1[ell] - O.s2_of(hh), gain, rel_tol=1e-12, abs_tol=1e-6), (ell, gain)


def test_s1_at_the_leaf_level_is_a_brute_force_count():
    # uniform scheme: the leaf neighbours of H_s are dense, so S1(L) counts the
    # entries (p, q) whose leaf boxes differ and are not standard-admissible
    P, k, eta, leaf = _case_2d(seed=3)
    tree = O.build_tree(P, leaf)
    hs = O.build(P, k, 1e-4, eta, tree.L, leaf, uniform=True)
    s1 = O.s1_by_level(hs)
    c = O.leaf_boxes(P, tree.L)                       # integer leaf-box coordinates
    uniq, inv, cnt = np.unique(c, axis=0, return_inverse=True, return_counts=True)
    count = 0
    for a in range(len(uniq)):
        for b in range(len(uniq)):
            if a != b and not O.adm_s(tuple(uniq[a]), tuple(uniq[b]), 2, eta):
                count += int(cnt[a]) * int(cnt[b])
    assert s1[tree.L] == float(count)


def test_walk_equals_brute_force_arg_max():
    P, k, eta, leaf = _case_2d()
    for uniform in (True, False):
        r = O.optimal_switch_level(P, k, 1e-6, eta, leaf, uniform=uniform)
        L = r["L"]
        gains = {L: 0.0}
        for ell in range(L):
            hh = O.build(P, k, 1e-6, eta, ell, leaf, uniform=uniform)
            gains[ell] = r["s1"][ell] - O.s2_of(hh)
        for ell, g in r["gains"].items():
            assert math.isclose(g, gains[ell], rel_tol=1e-12, abs_tol=1e-6)
        best = max(gains.values())
        # ties resolved towards the larger ell (the walk stops at a tie)
        assert r["ell"] == max(l for l, g in gains.items() if g == best), (gains, r["ell"])
        # eta = 1 in 2D leaves no admissible pair at level 1, so H_h(0) and
        # H_h(1) store the same blocks and the walk stops at 1 on the tie
        assert gains[0] == gains[1] and r["ell"] == 1


def test_hh_beats_hs_at_l_minus_1_in_3d():
    # Table tab:s1_s_2 (1/r in 3D, ell = L - 1): S1 > S2 at every eps, the
    # ratio larger at loose eps; same recipe at N = 4096, leaf 64 (L = 2)
    rng = np.random.default_rng(64)
    P = rng.uniform(-1.0, 1.0, (4096, 3))
    k = O.Kernel(W.INV_R)
    ratios = []
    for eps in (1e-2, 1e-6):
        hs = O.build(P, k, eps, math.sqrt(3), 2, 64, uniform=True)
        hh = O.build(P, k, eps, math.sqrt(3), 1, 64, uniform=True)
        ratios.append(O.s1_by_level(hs)[1] / O.s2_of(hh))
    assert all(r > 1.0 for r in ratios), ratios
    assert ratios[0] > ratios[1], ratios
