"""GPU parity of the switching-level choice (Sec. 3.3, Alg. 2) through the C
ABI: the library's walk against the oracle's on the same seeded points, in the
uniform and the mixed scheme. Both sides compress every block with the same
certified rule, so S1 and S2 agree up to the documented rank and format ties
(one tie moves a sum by one block's k (m + n) bits / 64); the walk's levels and
its result must be the same."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _compare(P, kind, eps, eta, leaf, uniform, mask=0xF):
    _torch()
    from paper_2604_09147_amd import switch_level_search
    print(f"switch level: n={P.shape[0]} d={P.shape[1]} eps={eps:g} uniform={uniform}", flush=True)
    g = switch_level_search(P, kind, eps, eta, leaf, mask=mask, uniform_fp64=uniform)
    o = O.optimal_switch_level(P, O.Kernel(kind), eps, eta, leaf, mask=mask, uniform=uniform)
    assert g["L"] == o["L"]
    assert g["ell"] == o["ell"], (g, o["gains"])
    assert np.allclose(g["s1"], o["s1"], rtol=2e-3, atol=0)
    walked = sorted(o["s2"])
    assert sorted(int(l) for l in np.flatnonzero(~np.isnan(g["s2"]))) == walked
    for l in walked:
        assert math.isclose(g["s2"][l], o["s2"][l], rel_tol=2e-3), (l, g["s2"][l], o["s2"][l])
    return g


@pytest.mark.parametrize("uniform", [True, False])
def test_switch_level_2d_matches_oracle(uniform):
    P = np.random.default_rng(7).random((2048, 2))
    g = _compare(P, W.INV_R, 1e-6, 1.0, 32, uniform)
    # eta = 1 leaves no admissible pair at level 1: H_h(0) = H_h(1), the walk
    # stops at 1 on the tie
    assert g["ell"] == 1 and g["s2"][0] == g["s2"][1]


def test_switch_level_3d_matches_oracle():
    P = np.random.default_rng(64).uniform(-1.0, 1.0, (4096, 3))
    _compare(P, W.INV_R, 1e-2, math.sqrt(3), 64, True)
