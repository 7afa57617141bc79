"""GPU parity with the FP64 oracle on the 3D benchmark recipe at N = 2^17.

Same recipe as the benchmark matrix (1/(4 pi r), points uniform in [0,1]^3 from
seed 303, leaf 256, eta 1.5, switching level L - 1, tol 1e-6, formats
{fp64, fp32, fp16, bf16}) at a size the oracle builds completely: L = 3 with
leaves of about 256 points, 2048 x 2048 interaction-list and neighbour blocks
(randomized compression) at the switching level and 256 x 256 siblings below
it (exact truncated SVD), as on the lower levels of the N = 2^20 matrix.

The oracle's matrix and products are stored in
tests/golden/oracle_3d_laplace_n131072.npz by make_oracle_reference.py (which
calls the oracle only). Checked: tree order, partition, every rank and every
format bit for bit (except decisions inside the tie windows of parity_util,
which are counted and listed), ||H~||^2 of Alg. 5, and H^ x, H^^T x (one and
16 right-hand sides) within 1e-2 tol of the oracle's products."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import format_window, rank_window, rel

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "oracle_3d_laplace_n131072.npz")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_headline_recipe_against_the_oracle():
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    ref = np.load(GOLD)
    n = int(ref["n"])
    p = W.cfg_3d_laplace(n=n, switch_level=-1)
    print(f"headline recipe N={n}: building on the GPU", flush=True)
    g = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale)
    st = g.stats()
    assert st["L"] == int(ref["L"]) == 3 and st["ell"] == int(ref["ell"]) == 2
    assert np.array_equal(g.perm(), O.build_tree(p.points, p.leaf_size).perm)
    bl = g.blocks()
    for key_g, key_o in (("level", "level"), ("box_i", "i"), ("box_j", "j"), ("kind", "kind"),
                         ("lowrank", "lowrank")):
        assert np.array_equal(bl[key_g].astype(ref[key_o].dtype), ref[key_o]), key_g
    # ranks: bit for bit outside the tie window of each block
    rank_ties = []
    for q in np.flatnonzero(bl["rank"] != ref["rank"]):
        w = rank_window(int(ref["pmin"][q]), int(ref["sketch"][q]), p.tol)
        thr = ref["thr"][q]
        near = [np.isfinite(t) and abs(t - thr) <= w * thr for t in (ref["tail"][q], ref["tail_prev"][q])]
        assert any(near) and abs(int(bl["rank"][q]) - int(ref["rank"][q])) == 1, \
            (q, bl["rank"][q], ref["rank"][q], ref["tail"][q], ref["tail_prev"][q], thr)
        rank_ties.append(int(q))
    # formats: bit for bit outside the tie window, on blocks of equal rank
    total2 = float(ref["total2"])
    fmt_ties = []
    nb = bl["level"].size
    for q in np.flatnonzero(bl["format"] != ref["fmt"]):
        if q in rank_ties:
            continue
        w = format_window(int(ref["rank"][q]), int(ref["pmin"][q]), nb)
        m = [O.format_margin(float(ref["nb2"][q]), total2, int(ref["level"][q]), 3, p.tol, f)
             for f in (W.FMT_BF16, W.FMT_FP16, W.FMT_FP32)]
        assert any(abs(v - 1.0) <= w for v in m), (q, bl["format"][q], ref["fmt"][q], m)
        fmt_ties.append(int(q))
    print(f"headline recipe: {nb} blocks, rank ties {rank_ties}, format ties {fmt_ties}", flush=True)
    assert len(rank_ties) + len(fmt_ties) <= max(3, nb // 1000)
    # Alg. 5 norm: the same sum over the blocks, in another order
    assert abs(st["norm2_total"] - total2) <= 1e-10 * total2
    # products against the oracle's
    x = np.random.default_rng(1).standard_normal(n)
    xd = torch.from_numpy(x).cuda()
    y = g.matvec(xd).cpu().numpy()
    yt = g.matvec_t(xd).cpu().numpy()
    e, et = rel(y, ref["y"]), rel(yt, ref["yt"])
    print(f"headline recipe: H x vs oracle {e:.2e}, H^T x vs oracle {et:.2e}", flush=True)
    assert e <= 1e-2 * p.tol and et <= 1e-2 * p.tol
    X = np.concatenate([x[:, None], np.random.default_rng(2).standard_normal((n, 15))], axis=1)
    Xd = torch.from_numpy(X).cuda()
    Y = g.matvec(Xd).cpu().numpy()
    YT = g.matvec_t(Xd).cpu().numpy()
    assert rel(Y[:, 0], ref["y"]) <= 1e-2 * p.tol and rel(YT[:, 0], ref["yt"]) <= 1e-2 * p.tol
    for r in (1, 15):
        y1 = g.matvec(Xd[:, r].contiguous()).cpu().numpy()
        assert rel(Y[:, r], y1) <= 1e-12
    g.free()
