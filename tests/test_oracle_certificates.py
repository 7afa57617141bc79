"""Pins for the parts of the oracle that smooth kernel matrices alone do not
exercise (each found by planting a mistake in a scratch copy of the oracle and
seeing no other test fail).

* Rank rule, Def. H_h(p, eps): the smallest k whose discarded tail is <=
  eps^2 ||H_b||^2, ties included (integer singular values make a tie exact).
* Randomized compression (R6) on a matrix with slowly decaying singular values,
  where the first sketch misses half the energy: the stored factors still meet
  ||H - U V^T||_F <= eps ||H||_F, and no rank below the exact-SVD minimum
  (Eckart-Young) is returned.
* Sign rule: the largest-magnitude entry of every U column is positive (first
  index on ties).
* Alg. 5: ||H~||^2 summed from the blocks equals the squared Frobenius norm of
  the assembled truncated matrix (blocks tile the matrix; U has orthonormal
  columns), which differs from ||H||^2 by about eps^2 at a loose eps.
* Transpose with a nonsymmetric kernel (double layer): H^^T x equals the
  transposed assembled matrix times x, diagonal blocks included.
* The leaf-neighbour storage test (Sec. 4.3) is strict at an exact tie."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O


def test_rank_rule_takes_an_exact_tie():
    # sigma = 7, 3, 1 x 6: ||H||^2 = 64; eps = 1/4 gives threshold 4, and the
    # tail after four values is exactly 4, so the rank is 4 (not 5)
    H = np.diag([7.0, 3.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    assert np.array_equal(np.linalg.svd(H, compute_uv=False), np.diag(H))
    c = O.compress(H, 0.25)
    assert c.thr == 4.0 and c.tail == 4.0 and c.rank == 4
    c = O.compress(H, 0.25 * (1 - 2 ** -20))
    assert c.rank == 5


@pytest.mark.parametrize("eps", [0.3, 0.5, 0.7])
def test_randomized_compression_is_certified_on_slow_decay(eps):
    rng = np.random.default_rng(0)
    H = rng.standard_normal((700, 560))             # flat spectrum: sketches miss energy
    c = O.compress(H, eps, 0, 7)
    assert c.sketch > 0                              # the randomized path ran
    err = np.linalg.norm(H - c.U @ c.V.T)
    assert err <= eps * np.linalg.norm(H) * (1 + 1e-12)
    sv = np.linalg.svd(H, compute_uv=False)
    tail = np.append(np.cumsum((sv ** 2)[::-1])[::-1], 0.0)
    k_min = int(np.argmax(tail <= eps * eps * np.sum(H * H)))
    assert c.rank >= k_min
    assert np.allclose(c.U.T @ c.U, np.eye(c.rank), atol=1e-12)


def test_sign_rule_on_every_column():
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((40, 30)),                       # exact SVD
            rng.standard_normal((700, 560)),                     # randomized
            O.dense_matrix(rng.random((200, 2)), O.Kernel(W.LOG))[:100, 100:]]
    for H in mats:
        c = O.compress(H, 0.3, 0, 11)
        assert c.rank > 0
        for r in range(c.rank):
            col = c.U[:, r]
            i = int(np.flatnonzero(np.abs(col) == np.abs(col).max())[0])
            assert col[i] > 0


@pytest.mark.parametrize("ell,uniform", [(-1, False), (1, False), (3, True)])
def test_alg5_norm_equals_the_assembled_truncated_matrix(ell, uniform):
    rng = np.random.default_rng(55)
    P = rng.random((900, 2))
    eps = 0.1
    hm = O.build(P, O.Kernel(W.INV_R), eps, 1.0, ell, 32, uniform=uniform)
    A, cover = O.assemble(hm, "truncated")
    assert cover.min() == 1 and cover.max() == 1
    assert math.isclose(float(np.sum(A * A)), hm.total2, rel_tol=1e-10)
    # the truncated norm sits measurably below the entry norm at this eps
    H = O.dense_matrix(P, O.Kernel(W.INV_R))
    assert hm.total2 < float(np.sum(H * H)) * (1 - 1e-6)


def test_transpose_with_the_nonsymmetric_double_layer_kernel():
    rng = np.random.default_rng(66)
    n = 700
    P = np.concatenate([W.sphere_surface(n // 2, 3, rng), W.ball_interior(n - n // 2, 3, rng)])
    nrm = W.unit_normals(n, 3, rng)
    k = O.Kernel(W.DOUBLE_LAYER, normals=nrm)
    hm = O.build(P, k, 1e-6, 1.5, -1, 16)
    A, _ = O.assemble(hm, "stored")
    assert np.linalg.norm(A - A.T) > 1e-3 * np.linalg.norm(A)       # really nonsymmetric
    diag_blocks = [sb.D for sb in hm.blocks if sb.blk.kind == O.T_DIAG and sb.D.shape[0] > 1]
    assert any(np.linalg.norm(D - D.T) > 1e-3 * np.linalg.norm(D) for D in diag_blocks)
    X = rng.standard_normal((n, 3))
    for got, want in ((O.matvec_t(hm, X), A.T @ X), (O.matvec(hm, X), A @ X)):
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_beneficial_storage_is_strict():
    # Sec. 4.3: factors replace a dense neighbour only when they take fewer
    # bits; at equality (rank 64 of a 64 x 64 block in fp32: 64 * 128 * 32 / 64
    # = 4096 words = 64 * 64) the block stays dense
    assert not O.beneficial(64, 64, 64, W.FMT_FP32)
    assert O.beneficial(63, 64, 64, W.FMT_FP32)
    assert not O.beneficial(128, 64, 64, W.FMT_BF16) and O.beneficial(127, 64, 64, W.FMT_BF16)


def test_global_bound_matches_the_printed_forms():
    # eq:error_bound_2d / eq:error_bound_3d (eta = sqrt d) for 1 <= ell <= L;
    # ell = 0 is the HODLR case, where C'' drops out
    for L in range(1, 7):
        for ell in range(1, L + 1):
            assert math.isclose(O.global_bound(2, math.sqrt(2), L, ell),
                                2 * math.sqrt(27 * ell + 8 + 3 * (L - ell)) + 1, rel_tol=1e-15)
            assert math.isclose(O.global_bound(3, math.sqrt(3), L, ell),
                                2 * math.sqrt(189 * ell + 26 + 7 * (L - ell)) + 1, rel_tol=1e-15)
        assert math.isclose(O.global_bound(3, math.sqrt(3), L, 0), 2 * math.sqrt(7 * L) + 1, rel_tol=1e-15)
    # the formula constants of eq:standard_IL_size / eq:standard_N_size at eta = sqrt d
    for d, want in ((2, (27, 8, 3)), (3, (189, 26, 7))):
        got = O.constants_formula(d, math.sqrt(d))
        assert all(math.isclose(g, w, rel_tol=1e-12) for g, w in zip(got, want)), (d, got)


def test_alg5_norm_does_not_depend_on_the_storage_decision():
    # with ell = L, Alg. 5 takes the leaf neighbours' norms from their entries
    # before Alg. 3 decides whether factors are stored: the mixed scheme (some
    # neighbours compressed) and the uniform one (all dense) share ||H~||^2
    rng = np.random.default_rng(77)
    P = rng.random((1500, 2))
    k = O.Kernel(W.INV_R)
    hm = O.build(P, k, 1e-3, math.sqrt(2), 4, 8)
    hu = O.build(P, k, 1e-3, math.sqrt(2), 4, 8, uniform=True)
    assert hm.ell == hm.tree.L == 4
    assert any(sb.lowrank and sb.blk.kind == O.T_DENSE_NEAR for sb in hm.blocks)
    assert hm.total2 == hu.total2
