"""GPU parity at the benchmark sizes, on samples the oracle computes one by one.

For the 3D Laplace matrix at N = 2^20 (the benchmark's configuration), the 2D
1/r matrix at N = 2^18 and the double-layer matrix at N = 2^19 (16 fp32
right-hand sides, transpose):

* the tree and the partition against the oracle's;
* 30 admissible blocks (one of every level and kind present, the largest
  level included, then random ones) compressed by the oracle: rank bit for
  bit outside the tie window, stored approximation within eps plus the
  format's rounding, and the format under the oracle's own estimate of
  ||H~||^2 (Lemma global_error puts ||H~|| within eps of ||H||). Row norms of
  a singular kernel are heavy-tailed, dominated by the closest pairs, so the
  estimate is the exact sum of H_ij^2 over every pair of points closer than
  rho (about 16 neighbours per point, found with a k-d tree) plus the part
  beyond rho from 2048 sampled rows, whose terms are bounded. A format is
  checked where the rule's decision is the same for every ||H~||^2 within a
  factor NORM2_SLACK of the estimate; the undecided blocks are counted.
  The N = 2^17 test of the same recipe checks every format against the
  oracle's exact ||H~||^2;
* the rows of two leaves against the fp64 product of the GPU's own exported
  factors;
* 2048 sampled rows of the product against the exact dense rows: relative
  2-norm over the sample <= 10 tol for the single-layer kernels; for the
  double layer, whose storage error the rule lets grow with the
  interaction-list constants, the bound of Thm amp_throrem with the
  enumerated constants (85.6 tol at L = 4, switching level 3, eta 1.5), with
  the 10 tol comparison and the largest per-row errors printed."""
import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import rank_window

pytestmark = pytest.mark.gpu

# Relative uncertainty allowed for the estimate of ||H~||^2: the sampled part
# (bounded terms, 2048 rows) is off by well under a percent at these sizes.
NORM2_SLACK = 1.05


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _structure(g, points, leaf, eta, ell):
    tree = O.build_tree(points, leaf)
    blocks = O.partition(tree, eta, ell)
    assert np.array_equal(g.perm(), tree.perm)
    bl = g.blocks()
    assert bl["level"].size == len(blocks)
    for key, attr in (("level", "level"), ("box_i", "i"), ("box_j", "j"), ("kind", "kind")):
        assert np.array_equal(bl[key], np.array([getattr(b, attr) for b in blocks])), key
    return tree, blocks, bl


def _dense_rows(points, kern, x, rows, trans, rho, chunk=64):
    """Exact rows of H x (of H^T x when trans) and, per row of H (column of H),
    the squared norm of its entries between points farther apart than rho,
    from the oracle's kernel entries."""
    n = points.shape[0]
    g = np.arange(n)
    x2 = x.reshape(n, -1)
    out = np.zeros((rows.size, x2.shape[1]))
    far2 = np.zeros(rows.size)
    sq = np.sum(points * points, axis=1)
    for a in range(0, rows.size, chunk):
        r = rows[a:a + chunk]
        if trans:
            nj = kern.normals[r] if kern.normals is not None else None
            blk = O.kernel_entries(kern, points, points[r], g, r, nj).T
        else:
            blk = O.kernel_entries(kern, points[r], points, r, g, kern.normals)
        out[a:a + chunk] = blk @ x2
        # squared distances through the Gram expansion (only compared with rho^2;
        # a pair within rounding of rho changes the sum by one bounded term)
        d2 = sq[r][:, None] + sq[None, :] - 2.0 * (points[r] @ points.T)
        far2[a:a + chunk] = np.sum(np.where(d2 > rho * rho, blk * blk, 0.0), axis=1)
    return out.reshape((rows.size,) + x.shape[1:]), far2


def _near_norm2(points, kern, rng, chunk=1 << 20):
    """rho (the median distance to the 16th nearest neighbour over 2048 sampled
    points) and the exact sum of H_ij^2 over every pair closer than rho. The
    entries of a singular kernel are largest there, so that what is left to
    estimate by sampling rows, the part beyond rho, has bounded terms."""
    from scipy.spatial import cKDTree
    n = points.shape[0]
    tree = cKDTree(points)
    d, _ = tree.query(points[rng.choice(n, 2048, replace=False)], k=17)
    rho = float(np.median(d[:, 16]))
    pairs = tree.query_pairs(rho, output_type="ndarray")
    near = 0.0
    nrm = kern.normals
    for a in range(0, pairs.shape[0], chunk):
        i, j = pairs[a:a + chunk, 0], pairs[a:a + chunk, 1]
        for u, v in ((i, j), (j, i)):
            e = O.kernel_pairs(kern, points[u], points[v], u, v, None if nrm is None else nrm[v])
            near += float(np.sum(e * e))
    return rho, near, pairs.shape[0]


def _sampled_blocks(g, kern, points, tree, blocks, bl, tol, rng, norm2_est, count=30):
    pt = points[tree.perm]
    nt = kern.normals[tree.perm] if kern.normals is not None else None
    lr = np.flatnonzero(bl["lowrank"].astype(bool))
    key = bl["level"][lr] * 8 + bl["kind"][lr]
    pick = [int(rng.choice(lr[key == k])) for k in np.unique(key)]
    rest = np.setdiff1d(lr, pick)
    pick += [int(q) for q in rng.choice(rest, max(count - len(pick), 0), replace=False)]
    undecided = 0
    for q in pick:
        b = blocks[q]
        H = O.block_entries(pt, kern, nt, b)
        c = O.compress(H, tol, 0, q)
        w = rank_window(min(b.m, b.n), c.sketch, tol)
        near = lambda t: np.isfinite(t) and abs(t - c.thr) <= w * c.thr
        assert bl["rank"][q] == c.rank or (abs(int(bl["rank"][q]) - c.rank) == 1 and (near(c.tail) or near(c.tail_prev))), \
            (q, bl["rank"][q], c.rank)
        if bl["rank"][q] == c.rank:
            nb2 = float(np.sum(c.sigma[:c.rank] ** 2))
            lo = O.choose_format(nb2, norm2_est / NORM2_SLACK, b.level, tree.d, tol, 0xF)
            hi = O.choose_format(nb2, norm2_est * NORM2_SLACK, b.level, tree.d, tol, 0xF)
            if lo == hi:
                assert bl["format"][q] == lo, (q, bl["format"][q], lo)
            else:
                undecided += 1
        U, V = g.block_factors(q)
        err = np.linalg.norm(H - U @ V.T) / max(np.linalg.norm(H), 1e-300)
        # eps ||H_b|| from the truncation plus the rounding of the stored
        # factors: ||U V^T - fl(U) fl(V)^T|| <= (2 u + u^2) sqrt(k) ||H~_b||
        # (orthonormal U, ||V||_F = ||H~_b||), with u of the block's format
        u = O.UNIT[int(bl["format"][q])]
        k = max(int(bl["rank"][q]), 1)
        assert err <= tol + 3.0 * u * np.sqrt(k), (q, err)
    print(f"  sampled blocks {len(pick)} (sizes up to {max(min(blocks[q].m, blocks[q].n) for q in pick)}), "
          f"formats undecided by the norm estimate: {undecided}", flush=True)
    assert undecided <= len(pick) // 5


def _leaf_rows_exported(g, bl, perm, x, leaves, trans=False):
    """Rows (tree order) of the chosen leaves of the fp64 product with the
    GPU's exported factors, and the matching caller indices."""
    xt = x[perm]
    key_lo, key_hi = ("col_begin", "col_end") if trans else ("row_begin", "row_end")
    oth_lo, oth_hi = ("row_begin", "row_end") if trans else ("col_begin", "col_end")
    out_rows, out_vals = [], []
    for (a, b) in leaves:
        y = np.zeros((b - a,) + xt.shape[1:])
        hit = np.flatnonzero((bl[key_lo] <= a) & (bl[key_hi] >= b))
        for q in hit:
            lo = int(bl[key_lo][q])
            jb, je = int(bl[oth_lo][q]), int(bl[oth_hi][q])
            A, B = g.block_factors(q)
            if bl["lowrank"][q]:
                if bl["rank"][q] == 0:
                    continue
                if trans:
                    A, B = B, A
                y += A[a - lo:b - lo] @ (B.T @ xt[jb:je])
            else:
                M = A.T if trans else A
                y += M[a - lo:b - lo] @ xt[jb:je]
        out_rows.append(perm[a:b])
        out_vals.append(y)
    return np.concatenate(out_rows), np.concatenate(out_vals)


def _leaves(g, bl, rng, count=2):
    L = g.stats()["L"]
    leaf = bl["level"] == L
    diag = np.flatnonzero(leaf & (bl["box_i"] == bl["box_j"]))
    q = rng.choice(diag, count, replace=False)
    return [(int(bl["row_begin"][i]), int(bl["row_end"][i])) for i in q]


def _run(problem, nrhs=1, io="f64", trans=False, seed=0, bar=None):
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    p = problem
    kern = O.Kernel(p.kernel, scale=p.scale, h=p.h, normals=p.normals)
    print(f"full size {p.name}: N={p.n}, building", flush=True)
    g = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                h=p.h, normals=p.normals, io_dtype=io)
    rng = np.random.default_rng(seed)
    tree, blocks, bl = _structure(g, p.points, p.leaf_size, p.eta, p.switch_level)
    print(f"full size {p.name}: structure matches", flush=True)
    shape = (p.n,) if nrhs == 1 else (p.n, nrhs)
    dt = torch.float32 if io == "f32" else torch.float64
    x = torch.from_numpy(rng.standard_normal(shape)).to(dt).cuda()
    y = (g.matvec_t(x) if trans else g.matvec(x)).double().cpu().numpy()
    xin = x.double().cpu().numpy()
    rows = rng.choice(p.n, 2048, replace=False)
    rho, near2, npairs = _near_norm2(p.points, kern, rng)
    yd, far2 = _dense_rows(p.points, kern, xin, rows, trans, rho)
    far_est = float(np.sum(far2)) * p.n / rows.size
    norm2_est = near2 + far_est
    print(f"full size {p.name}: ||H||^2 = {near2:.6e} (exact, {npairs} pairs closer than "
          f"{rho:.3e}) + {far_est:.6e} (2048 rows beyond) = {norm2_est:.6e}; sampling blocks",
          flush=True)
    _sampled_blocks(g, kern, p.points, tree, blocks, bl, p.tol, rng, norm2_est)
    r_idx, ye = _leaf_rows_exported(g, bl, g.perm(), xin, _leaves(g, bl, rng), trans)
    e_exp = np.linalg.norm(y[r_idx] - ye) / np.linalg.norm(ye)
    print(f"full size {p.name}: two leaves vs exported factors {e_exp:.2e}", flush=True)
    # fp64 arithmetic on the stored values (fp16/bf16 inner products in fp32 with
    # one RHS); fp32 outputs are rounded once more
    bound = 2.0 ** -22 if io == "f32" else (1e-12 if nrhs > 1 or not np.any(bl["format"] >= 2) else 1e-6)
    assert e_exp <= bound, (e_exp, bound)
    e_dense = np.linalg.norm(y[rows] - yd) / np.linalg.norm(yd)
    per_row = np.linalg.norm((y[rows] - yd).reshape(rows.size, -1), axis=1)
    ref_row = np.linalg.norm(yd.reshape(rows.size, -1), axis=1)
    top = np.sort(per_row)[::-1][:4] / np.linalg.norm(yd)
    worst = float(np.max(per_row / np.maximum(ref_row, 1e-300)))
    limit = max(10 * p.tol if bar is None else bar, 2.0 ** -22)
    print(f"full size {p.name}: 2048 sampled rows vs dense {e_dense:.2e} (bar {limit:.2e}, "
          f"10 tol {'met' if e_dense <= 10 * p.tol else 'missed'}); largest rows' share {top}; "
          f"largest per-row relative error {worst:.2e}", flush=True)
    assert e_dense <= limit
    g.free()


@pytest.mark.timeout(900)
def test_full_size_3d_laplace_headline():
    _run(W.cfg_3d_laplace(), seed=1)


@pytest.mark.timeout(900)
def test_full_size_2d_inv_r():
    _run(W.cfg_2d_inv_r(), seed=2)


@pytest.mark.timeout(900)
def test_full_size_double_layer_transpose_16_rhs():
    p = W.cfg_double_layer()
    # Thm amp_throrem with the enumerated constants of eta = 1.5 in 3D
    L = O.tree_depth(p.n, 3, p.leaf_size)
    c = O.global_bound(3, p.eta, L, O.resolve_switch_level(p.switch_level, L))
    _run(p, nrhs=16, io="f32", trans=True, seed=3, bar=c * p.tol)
