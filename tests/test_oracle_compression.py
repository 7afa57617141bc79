"""Pins of the oracle's compression (Sec. 2.2, Def. H_h(p, eps), reading R6) on
blocks shaped like the blocks of the benchmark matrices, against SVDs computed
by LAPACK drivers the oracle does not call (scipy's gesvd, or gesdd for
singular vectors).

* Blocks with min(m, n) <= 512 take the truncated SVD itself: the 256 x 256
  sibling blocks of the 3D benchmark (level 4, boxes of side 1/16 holding 256
  points each) get exactly the minimal rank of Eckart-Young.
* Larger blocks take the randomized range finder. On the benchmark's 2048 x
  2048 level-3 blocks (a face neighbour, rank about 300, and an interaction
  list block) and on a block of the nonsymmetric double-layer recipe, the
  randomized result is held to the exact one: its certified tail bounds its
  true error from above, Eckart-Young bounds that error from below, the rank
  is the exact minimal rank or one more, and the retained singular values
  agree with the exact ones (never above them, by interlacing).
* The double-layer block rounded to bf16 stays within eq:need_mvp."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import hh_oracle as O

EPS = 1e-6
SCALE = 1.0 / (4.0 * math.pi)


def _box_pair(n, side, offset, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n, 3)) * side
    b = (rng.random((n, 3)) + np.asarray(offset, dtype=float)) * side
    return a, b


def _laplace(a, b):
    m, n = a.shape[0], b.shape[0]
    return O.kernel_entries(O.Kernel(W.INV_R, scale=SCALE), a, b, np.arange(m),
                            np.arange(m, m + n), None)


def _minimal_rank(sv, thr):
    """Smallest k with sum_{r >= k} sv_r^2 <= thr, the tail summed from the
    smallest value up (sv from an independent LAPACK driver)."""
    tail = np.append(np.cumsum((sv ** 2)[::-1])[::-1], 0.0)
    return int(np.argmax(tail <= thr)), tail


@pytest.mark.parametrize("offset", [(1, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_sibling_blocks_take_the_exact_truncated_svd(offset):
    # face / edge / corner siblings of level 4 of the 3D benchmark
    a, b = _box_pair(256, 1.0 / 16.0, offset, seed=sum(offset))
    H = _laplace(a, b)
    c = O.compress(H, EPS, seed=303, uid=1)
    assert c.sketch == 0
    sv = scipy.linalg.svd(H, compute_uv=False, lapack_driver="gesvd")
    k, tail = _minimal_rank(sv, c.thr)
    assert c.rank == k
    assert tail[k] <= c.thr < tail[k - 1]
    err2 = float(np.sum((H - c.U @ c.V.T) ** 2))
    assert err2 <= c.thr * (1 + 1e-9)
    assert abs(err2 - tail[k]) <= 1e-9 * c.thr        # the optimum of Eckart-Young


def _randomized_against_exact(H, c):
    assert c.sketch > 0
    U, sv, Vt = scipy.linalg.svd(H, full_matrices=False, lapack_driver="gesdd")
    k, tail = _minimal_rank(sv, c.thr)
    # the certified tail adds ||H - Q Q^T H||^2 to the projected tail, so it can
    # only exceed the exact tail: rank never below the minimum, here at most one above
    assert c.rank in (k, k + 1), (c.rank, k)
    err2 = float(np.sum((H - c.U @ c.V.T) ** 2))
    assert tail[c.rank] * (1 - 1e-9) <= err2          # Eckart-Young lower bound
    assert err2 <= c.tail * (1 + 1e-9)                 # the certificate is an upper bound
    assert c.tail <= c.thr
    # retained singular values: interlacing keeps them at or below the exact ones,
    # one power iteration brings them within 1e-8 (relative to sigma_1)
    assert np.all(c.sigma <= sv[:c.rank] * (1 + 1e-12) + 1e-14 * sv[0])
    assert np.max(np.abs(c.sigma - sv[:c.rank])) <= 1e-8 * sv[0]
    # orthonormal left factor
    assert np.allclose(c.U.T @ c.U, np.eye(c.rank), atol=1e-12)
    return k


@pytest.mark.parametrize("offset", [(1, 0, 0), (2, 0, 0)])
def test_level3_blocks_randomized_against_exact_svd(offset):
    # 2048 points in boxes of side 1/8 (level 3 of the 3D benchmark): (1,0,0) is a
    # compressed face neighbour N_s at the switching level, (2,0,0) an IL_s block
    a, b = _box_pair(2048, 1.0 / 8.0, offset, seed=10 + offset[0])
    H = _laplace(a, b)
    c = O.compress(H, EPS, seed=303, uid=7 + offset[0])
    k = _randomized_against_exact(H, c)
    if offset == (1, 0, 0):
        assert k > 128 and c.sketch >= 256            # the wide-sketch rounds ran
    else:
        assert k < 48 and c.sketch == 64


def test_double_layer_block_randomized_and_bf16_rounding():
    # the nonsymmetric double-layer recipe at its full size (N = 2^19, half on the
    # unit sphere, half in the ball, random unit normals, leaf 256, L = 4): an
    # admissible pair of level-3 boxes of its tree, both above the exact-SVD size
    p = W.cfg_double_layer()
    P, nrm = p.points, p.normals
    tree = O.build_tree(P, p.leaf_size)
    assert tree.L == 4
    r3 = tree.ranges[3]
    sizes = r3[:, 1] - r3[:, 0]
    pick = None
    for i in np.argsort(-sizes):
        if not 600 <= sizes[i] <= 2500:
            continue
        ci = O.box_coords(int(i), 3, 3)
        for j in range(r3.shape[0]):
            cj = O.box_coords(j, 3, 3)
            if 600 <= sizes[j] <= 2500 and O.gap_S(ci, cj) <= 3 and O.adm_s(ci, cj, 3, p.eta):
                pick = (int(i), j)
                break
        if pick:
            break
    assert pick is not None
    (ib, ie), (jb, je) = tree.cluster(3, pick[0]), tree.cluster(3, pick[1])
    pt, nt = P[tree.perm], nrm[tree.perm]
    H = O.kernel_entries(O.Kernel(W.DOUBLE_LAYER, normals=nrm), pt[ib:ie], pt[jb:je],
                         np.arange(ib, ie), np.arange(jb, je), nt[jb:je])
    c = O.compress(H, EPS, seed=505, uid=3)
    _randomized_against_exact(H, c)
    # eq:need_mvp for the bf16 storage of this block's factors
    Hb = c.U @ c.V.T
    su, _, eu = O.quantize(c.U, W.FMT_BF16)
    sv_, _, ev = O.quantize(c.V, W.FMT_BF16)
    Hh = np.ldexp(su, eu) @ np.ldexp(sv_, ev).T
    u = O.UNIT[W.FMT_BF16]
    assert np.linalg.norm(Hb - Hh) <= (2.0 + math.sqrt(c.rank) * u) * u * np.linalg.norm(Hb)
