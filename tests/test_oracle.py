"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, closed forms, invariants, special cases that reduce to textbook
routines (a different SVD driver, brute force over all representable values),
and the paper's own error bounds."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import hh_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- tree (Sec. 2.1)
@pytest.mark.parametrize("n,d,leaf,L", [(262144, 2, 256, 5), (262144, 2, 64, 6),
                                        (64000, 3, 125, 3), (64000, 3, 64, 4)])
def test_tree_depth_matches_paper_examples(n, d, leaf, L):
    # (N, n_max, L) triples printed with the paper's storage experiments
    assert O.tree_depth(n, d, leaf) == L


@pytest.mark.parametrize("n,d,leaf", [(1, 2, 8), (37, 1, 4), (500, 2, 16), (777, 3, 8)])
def test_tree_boxes_contain_their_points(n, d, leaf):
    rng = np.random.default_rng(n)
    P = rng.random((n, d)) * 3.0 - 1.0
    t = O.build_tree(P, leaf)
    assert sorted(t.perm.tolist()) == list(range(n))
    lo = P.min(axis=0)
    side = float(np.max(P.max(axis=0) - lo)) or 1.0
    for level in range(t.L + 1):
        h = side / (1 << level)
        r = t.ranges[level]
        assert r[0, 0] == 0 and r[-1, 1] == n
        assert np.all(r[1:, 0] == r[:-1, 1])          # contiguous partition of [0, N)
        for box in range(r.shape[0]):
            b, e = r[box]
            if e == b:
                continue
            c = np.array(O.box_coords(box, level, d))
            pts = P[t.perm[b:e]]
            # geometric containment, with the top face of the cube closed
            assert np.all(pts >= lo + c * h - 1e-12 * side)
            assert np.all(pts <= lo + (c + 1) * h + 1e-12 * side)
            if level < t.L:                               # children nest in the parent
                ch = t.ranges[level + 1][box << d:(box + 1) << d]
                assert ch[0, 0] == b and ch[-1, 1] == e


def test_tree_membership_brute_force():
    # every point is in the level-l box floor(((p - lo) / side) 2^l), independently of Morton
    rng = np.random.default_rng(3)
    P = rng.random((300, 2))
    t = O.build_tree(P, 5)
    lo = P.min(axis=0)
    side = float(np.max(P.max(axis=0) - lo))
    for level in range(t.L + 1):
        c = np.minimum(np.floor(((P - lo) / side) * (1 << level)).astype(int), (1 << level) - 1)
        for box in range(1 << (2 * level)):
            b, e = t.ranges[level][box]
            want = {i for i in range(300) if tuple(c[i]) == O.box_coords(box, level, 2)}
            assert set(t.perm[b:e].tolist()) == want


# ---------------------------------------------------------- partition (Alg. 1)
def _full_lattice(d, L):
    """One point at the centre of every leaf box: every box of the tree is non-empty."""
    g = (np.arange(1 << L) + 0.5) / (1 << L)
    P = np.array(list(itertools.product(g, repeat=d)))
    return P


def _per_box_counts(blocks, level, kind):
    cnt = {}
    for b in blocks:
        if b.level == level and b.kind == kind:
            cnt[b.i] = cnt.get(b.i, 0) + 1
    return cnt


def test_fmm_list_sizes_2d():
    # eta = sqrt(2) reproduces the FMM lists: |IL_s| <= 27, |N_s| <= 8 (Sec. 2.3)
    P = _full_lattice(2, 5)
    t = O.build_tree(P, 1)
    assert t.L == 5
    bl = O.partition(t, math.sqrt(2.0), 4)
    il = _per_box_counts(bl, 4, O.T_FAR)
    ns = _per_box_counts(bl, 4, O.T_NEAR)
    assert max(il.values()) == 27 and max(ns.values()) == 8
    assert O.constants_enumerated(2, math.sqrt(2.0)) == (27, 8, 3)


def test_fmm_list_sizes_3d():
    # eq:error_bound_3d uses 189 and 26 for eta = sqrt(3)
    P = _full_lattice(3, 4)
    t = O.build_tree(P, 1)
    bl = O.partition(t, math.sqrt(3.0), 3)
    il = _per_box_counts(bl, 3, O.T_FAR)
    ns = _per_box_counts(bl, 3, O.T_NEAR)
    assert max(il.values()) == 189 and max(ns.values()) == 26
    assert O.constants_enumerated(3, math.sqrt(3.0)) == (189, 26, 7)


@pytest.mark.parametrize("d,eta", [(2, math.sqrt(2.0)), (3, math.sqrt(3.0))])
def test_formula_constants_equal_fmm_at_sqrt_d(d, eta):
    c1, c2, c3 = O.constants_formula(d, eta)
    want = {2: (27, 8, 3), 3: (189, 26, 7)}[d]
    assert abs(c1 - want[0]) < 1e-9 and abs(c2 - want[1]) < 1e-9 and c3 == want[2]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("factor", [1.0, 1.3, 2.0, 5.0])
def test_list_sizes_for_eta_at_least_sqrt_d(d, factor):
    # for eta >= sqrt(d) only touching boxes are inadmissible (S = 0), so
    # |N_s| = 3^d - 1 and |IL_s| = (2^d - 1) 3^d: a closed form independent of
    # the paper's bound formula (which is tight only at eta = sqrt(d))
    e1, e2, e3 = O.constants_enumerated(d, factor * math.sqrt(d))
    assert (e1, e2, e3) == ((2 ** d - 1) * 3 ** d, 3 ** d - 1, 2 ** d - 1)


def test_list_sizes_grow_as_eta_shrinks():
    sizes = [O.constants_enumerated(2, eta)[:2] for eta in (2.0, 1.0, 0.7, 0.5)]
    assert all(a[0] <= b[0] and a[1] <= b[1] for a, b in zip(sizes, sizes[1:]))


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_weak_list_is_siblings(d, L):
    # eq:weak_IL_size: |IL_w| = 2^d - 1 at every weak level (HODLR, ell = 0)
    t = O.build_tree(_full_lattice(d, L), 1)
    bl = O.partition(t, math.sqrt(d), 0)
    for level in range(1, L + 1):
        cnt = _per_box_counts(bl, level, O.T_WEAK)
        assert len(cnt) == 1 << (d * level)
        assert set(cnt.values()) == {2 ** d - 1}
    assert all(b.kind in (O.T_WEAK, O.T_DIAG) for b in bl)


def _tiling_ok(tree, blocks):
    n = tree.n
    cover = np.zeros((n, n), dtype=np.int32)
    for b in blocks:
        cover[b.ib:b.ie, b.jb:b.je] += 1
    return cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("n,d,leaf,eta,ell", [
    (300, 1, 8, 1.0, 2), (517, 2, 16, 1.0, 2), (517, 2, 16, math.sqrt(2), -1),
    (517, 2, 16, 2.0, 0), (517, 2, 16, 0.7, 3), (700, 3, 8, 1.5, 2),
    (700, 3, 8, math.sqrt(3), 3), (700, 3, 8, 1.5, 0)])
def test_partition_tiles_matrix_exactly_once(n, d, leaf, eta, ell):
    rng = np.random.default_rng(n + d)
    P = rng.random((n, d)) ** 2      # non-uniform density: empty boxes occur
    t = O.build_tree(P, leaf)
    bl = O.partition(t, eta, ell)
    assert _tiling_ok(t, bl)
    ellr = O.resolve_switch_level(ell, t.L)
    for b in bl:
        assert b.m > 0 and b.n > 0
        if b.kind == O.T_DIAG:
            assert b.level == t.L and b.i == b.j
        elif b.kind == O.T_FAR:
            assert b.level <= ellr
        elif b.kind in (O.T_NEAR, O.T_DENSE_NEAR):
            assert b.level == ellr and b.i != b.j
        else:
            assert b.level > ellr and (b.i >> d) == (b.j >> d)


def test_special_cases_hs_and_hodlr():
    # ell = L is the H_s matrix (dense leaf neighbours), ell = 0 is HODLR (Sec. 3.2)
    rng = np.random.default_rng(11)
    t = O.build_tree(rng.random((400, 2)), 8)
    hs = O.partition(t, math.sqrt(2), t.L)
    assert not any(b.kind in (O.T_WEAK, O.T_NEAR) for b in hs)
    assert any(b.kind == O.T_DENSE_NEAR for b in hs)
    hodlr = O.partition(t, math.sqrt(2), 0)
    assert {b.kind for b in hodlr} == {O.T_WEAK, O.T_DIAG}


# -------------------------------------------------------------- kernels (eq:kernel_mat)
def test_kernel_entries_closed_forms():
    pi = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0]])
    pj = np.array([[0.0, 0.0, 0.0]])
    gi, gj = np.array([0, 1]), np.array([5])
    nj = np.array([[0.0, 0.0, 1.0]])
    val = lambda kind, **kw: O.kernel_entries(O.Kernel(kind, **kw), pi, pj, gi, gj, nj)[:, 0]
    assert np.allclose(val(W.INV_R, scale=2.0), [2.0, 0.0])          # coincident -> 0
    assert np.allclose(val(W.INV_R2), [1.0, 0.0])
    assert np.allclose(val(W.LOG), [0.0, 0.0])
    assert np.allclose(val(W.GAUSS, h=1.0), [math.exp(-1.0), 1.0])   # regular at r = 0
    assert np.allclose(val(W.MATERN, h=0.5), [math.exp(-2.0), 1.0])
    assert np.allclose(val(W.DOUBLE_LAYER), [1.0, 0.0])
    p2 = np.array([[math.e, 0.0]])
    assert np.isclose(O.kernel_entries(O.Kernel(W.LOG), p2, np.zeros((1, 2)),
                                       np.array([0]), np.array([1]), None)[0, 0], 1.0)
    # diagonal of a singular kernel is zero
    P = np.random.default_rng(0).random((5, 2))
    assert np.all(np.diag(O.dense_matrix(P, O.Kernel(W.INV_R))) == 0.0)


# ----------------------------------------------------------- sketch generator
def test_splitmix64_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, k, out in rows:
        assert O.mix64((int(seed) + O.GAMMA * int(k)) & O.M64) == int(out)
    # the vectorised path agrees with the scalar path
    k = np.arange(1, 6, dtype=np.uint64)
    with np.errstate(over="ignore"):
        v = O.mix64(np.uint64(1234567) + np.uint64(O.GAMMA) * k)
    assert [int(a) for a in v] == [int(r[2]) for r in rows[1:]]


def test_sketch_is_balanced_rademacher():
    S = O.rademacher_sketch(42, 7, 0, 400, 32)
    assert set(np.unique(S)) == {-1.0, 1.0}
    assert abs(S.mean()) < 0.03
    assert np.abs(S.T @ S / 400 - np.eye(32)).max() < 0.3
    assert not np.array_equal(S, O.rademacher_sketch(42, 8, 0, 400, 32))


# --------------------------------------------------------- compression (Alg. 1)
def _block(m, n, seed=0, kind=W.INV_R, d=3, gap=1.0):
    rng = np.random.default_rng(seed)
    A = rng.random((m, d))
    B = rng.random((n, d)) + np.array([1.0 + gap] + [0.0] * (d - 1))
    return O.kernel_entries(O.Kernel(kind), A, B, np.arange(m), np.arange(m, m + n), None)


@pytest.mark.parametrize("eps,m,n", [(1e-2, 200, 150), (1e-6, 200, 150), (1e-10, 200, 150),
                                     (1e-6, 512, 300), (1e-8, 60, 50)])
def test_exact_compression_rank_is_minimal(eps, m, n):
    # Eckart-Young with an independent LAPACK driver: the rank-(k-1) optimum misses eps
    H = _block(m, n, 1, gap=0.2)
    c = O.compress(H, eps)
    assert c.sketch == 0
    s = scipy.linalg.svd(H, compute_uv=False, lapack_driver="gesvd")
    nrm = np.linalg.norm(H)
    err = np.linalg.norm(H - c.U @ c.V.T)
    assert err <= eps * nrm * (1 + 1e-6)
    assert math.sqrt(np.sum(s[c.rank - 1:] ** 2)) > eps * nrm
    assert np.allclose(c.U.T @ c.U, np.eye(c.rank), atol=1e-12)


@pytest.mark.parametrize("eps,m,n", [(1e-4, 700, 640), (1e-8, 700, 640), (1e-6, 600, 520),
                                     (1e-10, 530, 1100)])
def test_randomized_compression_matches_exact_rank(eps, m, n):
    # block above the exact-SVD size: the certified bound holds and the rank equals
    # the rank of the exact SVD computed by an independent LAPACK driver
    H = _block(m, n, 2, gap=0.5)
    c = O.compress(H, eps, seed=9, uid=3)
    assert c.sketch > 0
    nrm2 = float(np.sum(H * H))
    err2 = float(np.sum((H - c.U @ c.V.T) ** 2))
    assert err2 <= (eps * eps) * nrm2 * (1 + 1e-6)
    s = scipy.linalg.svd(H, compute_uv=False, lapack_driver="gesvd")
    tails = np.cumsum((s ** 2)[::-1])[::-1]
    k_exact = int(np.argmax(np.append(tails, 0.0) <= (eps * eps) * nrm2))
    assert c.rank == k_exact
    assert np.allclose(c.U.T @ c.U, np.eye(c.rank), atol=1e-12)


def test_zero_block_has_rank_zero():
    c = O.compress(np.zeros((10, 7)), 1e-6)
    assert c.rank == 0 and c.U.shape == (10, 0)


# ------------------------------------------------------------ rounding (R8)
def _all_fp16():
    v = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16).astype(np.float64)
    return np.unique(v[np.isfinite(v)])


def _nearest_even(x, grid, bits_of):
    i = np.searchsorted(grid, x)
    lo, hi = grid[max(i - 1, 0)], grid[min(i, grid.size - 1)]
    dl, dh = abs(x - lo), abs(hi - x)
    if dl < dh:
        return lo
    if dh < dl:
        return hi
    return lo if bits_of(lo) % 2 == 0 else hi


def test_fp16_rounding_brute_force():
    grid = _all_fp16()
    bits = lambda v: int(np.float16(v).view(np.uint16))
    rng = np.random.default_rng(5)
    xs = list(rng.standard_normal(300) * 10.0 ** rng.integers(-7, 5, 300))
    mids = (grid[1:] + grid[:-1]) / 2.0                 # exact ties
    xs += list(rng.choice(mids[np.abs(mids) < 6e4], 300))
    for x in xs:
        assert float(np.float64(x).astype(np.float16)) == _nearest_even(x, grid, bits)


def test_bf16_rounding_brute_force():
    rng = np.random.default_rng(6)
    xs = list(rng.standard_normal(400) * 10.0 ** rng.integers(-40, 30, 400))
    bits = lambda v: int(np.float32(v).view(np.uint32) >> 16)
    for x in xs:
        # all bf16 magnitudes near |x|: patterns adjacent to the truncated pattern
        ax = abs(x)
        b = int(np.float32(ax).view(np.uint32) >> 16)
        cand = np.array([max(b + o, 0) for o in (-1, 0, 1, 2)], dtype=np.uint32) << 16
        vals = np.unique(cand.view(np.float32).astype(np.float64))
        got = float(O.round_bf16(np.array([x]))[0])
        assert got == math.copysign(_nearest_even(ax, vals, bits), x)
    # an exact tie between two bf16 neighbours rounds to the even pattern
    lo = np.array([0x3F80], dtype=np.uint32) << 16     # 1.0
    tie = float(lo.view(np.float32)[0]) + 2.0 ** -8
    assert float(O.round_bf16(np.array([tie]))[0]) == 1.0


@pytest.mark.parametrize("fmt,lo,hi", [(W.FMT_FP16, 2.0 ** 14, 2.0 ** 15), (W.FMT_BF16, 1.0, 2.0)])
def test_scaling_puts_max_in_range(fmt, lo, hi):
    rng = np.random.default_rng(8)
    for mag in (1e-30, 1e-3, 1.0, 7e4, 1e20):
        F = rng.standard_normal((30, 4)) * mag
        e = O.scale_exponent(F, fmt)
        mx = np.max(np.abs(np.ldexp(F, -e)))
        assert lo <= mx < hi


# ----------------------------------------------------- precision rule (Alg. 3)
def test_precision_rule_thresholds_and_ties():
    d, level, eps, total2 = 3, 2, 1e-4, 1.0
    # u^2 2^(dl) nb2 <= eps^2 total2 ; exact tie for bf16 when nb2 = eps^2 / (u^2 2^(dl))
    nb2_tie = (eps * eps) / ((2.0 ** -16) * 2.0 ** 6)
    assert O.choose_format(nb2_tie, total2, level, d, eps, 0xF) == W.FMT_BF16
    assert O.choose_format(nb2_tie * (1 + 2 ** -40), total2, level, d, eps, 0xF) == W.FMT_FP16
    # bf16 is the lowest precision, so it wins over fp16 when both qualify
    assert O.choose_format(nb2_tie / 4, total2, level, d, eps, 0xF) == W.FMT_BF16
    assert O.choose_format(nb2_tie / 4, total2, level, d, eps, 0x7) == W.FMT_FP16
    assert O.choose_format(1.0, total2, level, d, 1e-4, 0xF) == W.FMT_FP32   # 2^-42 <= 1e-8
    assert O.choose_format(1.0, total2, level, d, 1e-9, 0xF) == W.FMT_FP64   # 2^-42 > 1e-18
    assert O.choose_format(1e-9, total2, level, d, eps, 0x1) == W.FMT_FP64


def test_beneficial_worked_example():
    # 125 x 125 neighbour with rank 64 (Sec. 4.3): fp64 not worth it, fp32 is
    assert not O.beneficial(64, 125, 125, W.FMT_FP64)
    assert O.beneficial(64, 125, 125, W.FMT_FP32)


# ------------------------------------------- construction, mat-vec and bounds
def _problem(n=1500, d=2, kind=W.LOG, leaf=32, eps=1e-6, eta=1.0, ell=-1, seed=21, dom=1.0):
    rng = np.random.default_rng(seed)
    P = rng.random((n, d)) * dom
    return P, O.Kernel(kind), eps, eta, ell, leaf


@pytest.fixture(scope="module", params=[(1e-6, 0xF), (1e-3, 0xF), (1e-3, 0x7)],
                ids=["fp32", "fp16+bf16", "fp16"])
def small_h(request):
    eps, mask = request.param
    P, k, _, eta, ell, leaf = _problem()
    hm = O.build(P, k, eps, eta, ell, leaf, mask=mask)
    H = O.dense_matrix(P, k)
    return hm, H


def test_lemma_global_error_uniform():
    # Lemma global_error: ||H - H~|| <= eps ||H||, blockwise and globally
    for ell in (0, 1, 2, 3):
        P, k, eps, eta, _, leaf = _problem(n=1200, eps=1e-5, seed=ell)
        hm = O.build(P, k, eps, eta, ell, leaf, uniform=True)
        H = O.dense_matrix(P, k)
        A, cover = O.assemble(hm, "truncated")
        assert cover.min() == 1 and cover.max() == 1
        assert np.linalg.norm(H - A) <= eps * np.linalg.norm(H) * (1 + 1e-6)


def test_block_rounding_bound(small_h):
    # eq:need_mvp: ||H~_b - H^_b|| <= (2 + sqrt(p) u_b) u_b ||H~_b|| for every block
    hm, _ = small_h
    for sb in hm.blocks:
        if sb.lowrank and sb.rank:
            u = O.UNIT[sb.fmt]
            d = np.linalg.norm(sb.Ut @ sb.Vt.T - sb.U @ sb.V.T)
            assert d <= (2 + math.sqrt(sb.rank) * u) * u * math.sqrt(sb.nb2) * (1 + 1e-9)


def test_global_mixed_precision_bound(small_h):
    # Thm amp_throrem with the enumerated sparsity constants
    hm, H = small_h
    A, _ = O.assemble(hm, "stored")
    c = O.global_bound(hm.d, hm.eta, hm.tree.L, hm.ell)
    assert np.linalg.norm(H - A) <= c * hm.eps * np.linalg.norm(H)
    fm = O.storage(hm)["blocks_by_format"]
    want = {1e-6: {W.FMT_FP32}, 1e-3: {W.FMT_FP16, W.FMT_BF16} if hm.mask == 0xF else {W.FMT_FP16}}
    assert {f for f, c in fm.items() if c} == want[hm.eps]


@pytest.mark.parametrize("ell", [0, 3, 4])
def test_special_case_bounds(ell):
    # ell = 0 (HODLR) and ell = L (H_s, eq:err2_bound) in adaptive precision
    P, k, eps, eta, _, leaf = _problem(n=1100, eps=1e-4, seed=40 + ell, kind=W.INV_R, leaf=8)
    hm = O.build(P, k, eps, eta, ell, leaf, mask=0xF)
    assert hm.tree.L == 4
    H = O.dense_matrix(P, k)
    A, cover = O.assemble(hm, "stored")
    assert cover.min() == 1 and cover.max() == 1
    c = O.global_bound(hm.d, hm.eta, hm.tree.L, hm.ell)
    assert np.linalg.norm(H - A) <= c * eps * np.linalg.norm(H)


def test_matvec_equals_assembled_matrix(small_h):
    # Alg. 4 block by block equals the product with the assembled H^
    hm, H = small_h
    A, _ = O.assemble(hm, "stored")
    x = np.random.default_rng(2).standard_normal((hm.n, 3))
    y = O.matvec(hm, x)
    assert np.linalg.norm(y - A @ x) <= 1e-13 * np.linalg.norm(A @ x)
    yt = O.matvec_t(hm, x)
    assert np.linalg.norm(yt - A.T @ x) <= 1e-13 * np.linalg.norm(A.T @ x)
    # adjoint identity <w, H^ v> = <H^T w, v>
    v, w = x[:, 0], x[:, 1]
    assert abs(w @ O.matvec(hm, v) - O.matvec_t(hm, w) @ v) <= 1e-12 * abs(w @ (A @ v)) + 1e-12


def test_matvec_backward_error(small_h):
    # Thm mvp with x ~ U(0, 1) as in Sec. 5.3
    hm, H = small_h
    x = np.random.default_rng(3).random(hm.n)
    b = O.matvec(hm, x)
    c = O.global_bound(hm.d, hm.eta, hm.tree.L, hm.ell)
    assert np.linalg.norm(H @ x - b) / (np.linalg.norm(H) * np.linalg.norm(x)) <= 2 * c * hm.eps


def test_dense_matvec_helpers():
    P, k, *_ = _problem(n=300, kind=W.DOUBLE_LAYER, d=3)
    k = O.Kernel(W.DOUBLE_LAYER, normals=W.unit_normals(300, 3, np.random.default_rng(1)))
    H = O.dense_matrix(P, k)
    assert not np.allclose(H, H.T)
    x = np.random.default_rng(4).standard_normal(300)
    assert np.allclose(O.dense_matvec(P, k, x, chunk=64), H @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(O.dense_matvec_t(P, k, x, chunk=64), H.T @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(O.dense_matvec(P, k, x, rows=np.array([3, 7])), (H @ x)[[3, 7]])


def test_fp64_only_for_tight_tolerances():
    # Sec. 5.2: for 1e-12 <= eps <= 1e-10 the adaptive scheme keeps fp64 only
    rng = np.random.default_rng(12)
    P = rng.random((2000, 2)) * 2.0 - 1.0
    for eps in (1e-12, 1e-10):
        hm = O.build(P, O.Kernel(W.LOG), eps, math.sqrt(2.0), -1, 32, mask=0xF)
        fm = O.storage(hm)["blocks_by_format"]
        assert fm[W.FMT_FP32] == fm[W.FMT_FP16] == fm[W.FMT_BF16] == 0
