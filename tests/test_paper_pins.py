"""The values the paper prints (tests/golden/paper_pins.txt), each recomputed
from the oracle and compared with the fixture's text."""
import math
import os

import numpy as np

import workloads as W
from oracle import hh_oracle as O

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_pins.txt")


def _entries():
    # fields are separated by " | "; a value may itself contain bars (|IL_s|)
    # but never a bar with a space on both sides
    out = {}
    for line in open(FIXTURE):
        if line.startswith("#") or not line.strip():
            continue
        fields = line.rstrip("\n").split(" | ")
        assert len(fields) == 3, line
        name, value, where = (f.strip() for f in fields)
        out[name] = (value, where)
    return out


def _tree(n, d, leaf):
    return f"L={O.tree_depth(n, d, leaf)}"


def _fmm_counts():
    c1, c2, _ = O.constants_enumerated(2, math.sqrt(2))
    return f"|IL_s| <= {c1}, |N_s| <= {c2}"


def _fmm_bound(d):
    c1, c2, c3 = O.constants_enumerated(d, math.sqrt(d))
    return f"{c1} l + {c2} + {c3} (L - l)"


def _weak_il():
    # the open pairs below the switching level are the 2^d - 1 siblings of a box
    for d in (1, 2, 3):
        rng = np.random.default_rng(d)
        tree = O.build_tree(rng.random((64 ** d if d < 3 else 4096, d)), 8)
        blocks = O.partition(tree, math.sqrt(d), 0)
        per_box = {}
        for b in blocks:
            if b.kind == O.T_WEAK:
                per_box[(b.level, b.i)] = per_box.get((b.level, b.i), 0) + 1
        assert max(per_box.values()) == 2 ** d - 1
    return "|IL_w| = 2^d - 1"


def _q43_range():
    xmin = 2.0 ** O.Q43_EMIN
    xmax = float(O.round_q43(np.array([240.0]))[0])
    assert O.round_q43(np.array([xmin]))[0] == xmin and np.isinf(O.round_q43(np.array([248.0]))[0])
    return f"x_min={xmin:.2e} x_max={xmax:.2e} e_min={O.Q43_EMIN} e_max={O.Q43_EMAX}"


def _xmax_bf16():
    top = float(O.round_bf16(np.array([3.39e38]))[0])
    assert np.isfinite(top) and np.isinf(O.round_bf16(np.array([3.41e38]))[0])
    return f"{top:.2e}"


def _beneficial():
    assert not O.beneficial(64, 125, 125, W.FMT_FP64) and O.beneficial(64, 125, 125, W.FMT_FP32)
    return "rank 64, 125 x 125: fp64 not beneficial, fp32 beneficial"


def _fp64_only():
    rng = np.random.default_rng(12)
    P = rng.random((700, 2)) * 2.0 - 1.0
    for eps in (1e-12, 1e-10):
        hm = O.build(P, O.Kernel(W.LOG), eps, math.sqrt(2.0), -1, 16, mask=0xF)
        fm = O.storage(hm)["blocks_by_format"]
        assert sum(c for f, c in fm.items() if f != W.FMT_FP64) == 0
    return "1e-12 <= eps <= 1e-10 gives fp64 only"


def _s1_over_s2():
    rng = np.random.default_rng(64)
    P = rng.uniform(-1.0, 1.0, (4096, 3))
    k = O.Kernel(W.INV_R)
    hs = O.build(P, k, 1e-2, math.sqrt(3), 2, 64, uniform=True)
    hh = O.build(P, k, 1e-2, math.sqrt(3), 1, 64, uniform=True)
    assert O.s1_by_level(hs)[1] > O.s2_of(hh)
    return "S1/S2 > 1 at ell = L - 1"


CHECKS = {
    "tree_2d_262144_256": lambda: _tree(262144, 2, 256),
    "tree_2d_262144_64": lambda: _tree(262144, 2, 64),
    "tree_3d_64000_125": lambda: _tree(64000, 3, 125),
    "tree_3d_64000_64": lambda: _tree(64000, 3, 64),
    "tree_2d_6400": lambda: _tree(6400, 2, 25),
    "fmm_2d_sqrt2": _fmm_counts,
    "fmm_3d_sqrt3": lambda: _fmm_bound(3),
    "fmm_2d_bound": lambda: _fmm_bound(2),
    "weak_il": _weak_il,
    "unit_fp64": lambda: f"{O.UNIT[W.FMT_FP64]:.2e}",
    "unit_fp32": lambda: f"{O.UNIT[W.FMT_FP32]:.2e}",
    "unit_fp16": lambda: f"{O.UNIT[W.FMT_FP16]:.2e}",
    "unit_bf16": lambda: f"{O.UNIT[W.FMT_BF16]:.2e}",
    "xmax_bf16": _xmax_bf16,
    "q43_range": _q43_range,
    "beneficial_125": _beneficial,
    "fp64_only": _fp64_only,
    "s1_over_s2_3d": _s1_over_s2,
}


def test_every_fixture_line_has_a_check():
    assert set(_entries()) == set(CHECKS)


def test_printed_values_match_the_oracle():
    for name, (value, where) in _entries().items():
        assert CHECKS[name]() == value, (name, where)
