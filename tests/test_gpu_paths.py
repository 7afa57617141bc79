"""GPU tests of the differentiable product (transpose as backward), the
batched launch over many handles and handles derived from a uniform fp64 one,
all through the C ABI.

Bars as in the parity tests: 1e-2 tol (relative 2-norm) against the oracle's
own H^ product, 10 tol against the dense kernel product, with the fp32 io
floor 2^-22 for fp32 inputs and outputs."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hh_oracle as O
from parity_util import build_pair, compare_structure, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _double_layer_problem(n, seed):
    rng = np.random.default_rng(seed)
    P = np.concatenate([W.sphere_surface(n // 2, 3, rng), W.ball_interior(n - n // 2, 3, rng)])
    return P, W.unit_normals(n, 3, rng)


def test_autograd_backward_is_the_transposed_product():
    # nonsymmetric double-layer kernel, sphere + ball, 16 fp32 right-hand sides
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    from paper_2604_09147_amd.autograd import hh_apply
    tol = 1e-6
    P, nrm = _double_layer_problem(3000, 505)
    g, o = build_pair(P, W.DOUBLE_LAYER, tol, 1.5, -1, 64, normals=nrm, io="f32")
    compare_structure(g, o)
    rng = np.random.default_rng(7)
    x = torch.from_numpy(rng.standard_normal((3000, 16))).float().cuda().requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((3000, 16))).float().cuda()
    y = hh_apply(g, x)
    (y * w).sum().backward()
    grad = x.grad.double().cpu().numpy()
    wd = w.double().cpu().numpy()
    k = O.Kernel(W.DOUBLE_LAYER, normals=nrm)
    bar = max(1e-2 * tol, 2.0 ** -22)
    assert rel(grad, O.matvec_t(o, wd)) <= bar
    assert rel(grad, O.dense_matvec_t(P, k, wd)) <= 10 * tol
    # the forward pass is the product itself
    assert rel(y.detach().double().cpu().numpy(), O.matvec(o, x.detach().double().cpu().numpy())) <= bar

    # finite differences of f(x) = <w, H^ x> in fp64 (step 1e-3): with fp64 /
    # fp32 storage the product is computed in fp64, f is linear, and the
    # central difference equals <H^T w, e> up to rounding
    g64 = HMatrix(P, W.DOUBLE_LAYER, tol, 1.5, -1, 64, normals=nrm, mask=0x3)
    x64 = torch.from_numpy(rng.standard_normal(3000)).cuda()
    w64 = torch.from_numpy(rng.standard_normal(3000)).cuda()
    xr = x64.clone().requires_grad_(True)
    (hh_apply(g64, xr) * w64).sum().backward()
    for t in range(3):
        e = torch.from_numpy(rng.standard_normal(3000)).cuda()
        h = 1e-3
        fp = float((g64.matvec(x64 + h * e) * w64).sum())
        fm = float((g64.matvec(x64 - h * e) * w64).sum())
        fd = (fp - fm) / (2 * h)
        an = float((xr.grad * e).sum())
        assert abs(fd - an) <= 1e-9 * max(abs(an), 1.0), (fd, an)
    g64.free()


def _assembled_gpu_matrix(g):
    """Dense N x N matrix (caller order) from the GPU's stored, decoded blocks."""
    n = g.n
    perm = g.perm()
    bl = g.blocks()
    A = np.zeros((n, n))
    for q in range(bl["level"].size):
        ri = perm[int(bl["row_begin"][q]):int(bl["row_end"][q])]
        cj = perm[int(bl["col_begin"][q]):int(bl["col_end"][q])]
        U, V = g.block_factors(q)
        if bl["lowrank"][q]:
            if bl["rank"][q]:
                A[np.ix_(ri, cj)] += U @ V.T
        else:
            A[np.ix_(ri, cj)] += U
    return A


def test_double_layer_4096_point_subsample_against_dense_transpose():
    # the double-layer recipe's own check: an H_h built on 4096 points drawn from
    # the N = 2^19 recipe (same kernel and normals, tol 1e-6, eta 1.5, leaf 256,
    # switching level L - 1), 16 fp32 right-hand sides through autograd; the
    # backward pass against the dense fp64 transpose on all 4096 rows
    torch = _torch()
    from paper_2604_09147_amd.autograd import hh_apply
    p = W.cfg_double_layer()
    idx = np.random.default_rng(5050).choice(p.n, 4096, replace=False)
    P, nrm = p.points[idx], p.normals[idx]
    g, o = build_pair(P, W.DOUBLE_LAYER, p.tol, p.eta, -1, p.leaf_size, normals=nrm, io="f32")
    compare_structure(g, o)
    k = O.Kernel(W.DOUBLE_LAYER, normals=nrm)
    Hd = O.dense_matrix(P, k)
    # Thm amp_throrem on the stored matrix, enumerated constants of eta = 1.5
    c = O.global_bound(3, p.eta, o.tree.L, o.ell)
    e_mat = np.linalg.norm(Hd - _assembled_gpu_matrix(g)) / np.linalg.norm(Hd)
    assert e_mat <= c * p.tol, (e_mat, c)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal((4096, 16))).float().cuda().requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((4096, 16))).float().cuda()
    (hh_apply(g, x) * w).sum().backward()
    grad = x.grad.double().cpu().numpy()
    ref = Hd.T @ w.double().cpu().numpy()
    e = rel(grad, ref)
    per_row = np.linalg.norm(grad - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"double layer, 4096-point subsample (L={o.tree.L}, switching level {o.ell}): "
          f"||H - H^||_F / ||H||_F = {e_mat:.2e} (Thm amp bound {c * p.tol:.2e}); backward vs "
          f"dense transpose {e:.2e} (10 tol {'met' if e <= 10 * p.tol else 'missed'}), largest "
          f"per-row relative error {per_row.max():.2e}", flush=True)
    assert e <= max(c * p.tol, 2.0 ** -22)
    assert rel(grad, O.matvec_t(o, w.double().cpu().numpy())) <= max(1e-2 * p.tol, 2.0 ** -22)


def test_transpose_adjoint_identity():
    # <w, H^ x> = <H^^T w, x> with the same stored factors (fp64 arithmetic)
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    P, nrm = _double_layer_problem(5000, 11)
    g = HMatrix(P, W.DOUBLE_LAYER, 1e-6, 1.5, -1, 64, normals=nrm, mask=0x3)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal(5000)).cuda()
    w = torch.from_numpy(rng.standard_normal(5000)).cuda()
    a = float((w * g.matvec(x)).sum())
    b = float((g.matvec_t(w) * x).sum())
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0), (a, b)
    g.free()


def test_batched_launch_equals_individual_products():
    # uneven instances of the batched workload: Gaussian kernels, log-uniform
    # sizes, mixed tolerances, fp32 io; one launch per phase over all handles
    torch = _torch()
    from paper_2604_09147_amd import HMatrix, matvec_batch
    rng = np.random.default_rng(404)
    mats, xs, probs = [], [], []
    for t in range(6):
        n = int(2 ** rng.uniform(10, 13))
        P = rng.random((n, 3))
        h = float(rng.uniform(0.05, 0.3))
        tol = float(rng.choice([1e-4, 1e-6, 1e-8]))
        m = HMatrix(P, W.GAUSS, tol, math.sqrt(3), -1, 64, h=h, io_dtype="f32")
        mats.append(m)
        probs.append((P, h, tol))
        xs.append(torch.from_numpy(rng.standard_normal(n)).float().cuda())
    ys = matvec_batch(mats, xs)
    torch.cuda.synchronize()
    for m, x, y in zip(mats, xs, ys):
        yi = m.matvec(x)
        assert torch.equal(y, yi), "batched product differs from the single product"
    # the smallest instance against the oracle and the dense product
    i = int(np.argmin([p[0].shape[0] for p in probs]))
    P, h, tol = probs[i]
    o = O.build(P, O.Kernel(W.GAUSS, h=h), tol, math.sqrt(3), -1, 64)
    compare_structure(mats[i], o)
    xin = xs[i].double().cpu().numpy()
    y = ys[i].double().cpu().numpy()
    bar = max(1e-2 * tol, 2.0 ** -22)
    assert rel(y, O.matvec(o, xin)) <= bar
    assert rel(y, O.dense_matvec(P, O.Kernel(W.GAUSS, h=h), xin)) <= max(10 * tol, 2.0 ** -22)
    for m in mats:
        m.free()


def test_derived_handle_equals_direct_build():
    # Alg. 3 applied to the fp64 factors of a uniform handle gives the handle a
    # direct adaptive build gives (same tree, partition, ranks, formats, rounding)
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    rng = np.random.default_rng(21)
    P = rng.random((6000, 3))
    g64 = HMatrix(P, W.INV_R, 1e-5, 1.5, -1, 64, uniform_fp64=True)
    ga = g64.derive(mask=0xF)
    gd = HMatrix(P, W.INV_R, 1e-5, 1.5, -1, 64)
    ba, bd = ga.blocks(), gd.blocks()
    for key in ("level", "box_i", "box_j", "rank", "format"):
        assert np.array_equal(ba[key], bd[key]), key
    assert np.all(g64.blocks()["format"][g64.blocks()["lowrank"].astype(bool)] == W.FMT_FP64)
    x = torch.from_numpy(rng.standard_normal(6000)).cuda()
    ya, yd = ga.matvec(x), gd.matvec(x)
    assert float(torch.linalg.norm(ya - yd) / torch.linalg.norm(yd)) <= 1e-15
    y64 = g64.matvec(x)
    assert float(torch.linalg.norm(ya - y64) / torch.linalg.norm(y64)) <= 1e-5
    for m in (ga, gd, g64):
        m.free()


def test_runs_cut_at_a_lowered_buffer_limit(monkeypatch):
    # The accumulation kernels address each run of factor columns through one
    # buffer descriptor (32-bit byte offsets), so hh_build cuts runs and their
    # work-unit slices below 2^31 bytes. Lowering that limit to 64 KiB makes
    # the cutting happen at this size: products must not change.
    torch = _torch()
    from paper_2604_09147_amd import HHError, HMatrix
    p = W.cfg_plain_small(seed=5, n=3000)
    tol = 1e-6
    _, o = build_pair(p.points, p.kernel, tol, p.eta, -1, 48)
    monkeypatch.setenv("HH_RUN_BYTES_MAX", "65536")
    g = HMatrix(p.points, p.kernel, tol, p.eta, -1, 48)
    compare_structure(g, o)
    rng = np.random.default_rng(21)
    for nrhs in (1, 5):
        x = rng.standard_normal((3000, nrhs))
        xd = torch.from_numpy(x).cuda()
        assert rel(g.matvec(xd).cpu().numpy(), O.matvec(o, x)) <= 1e-2 * tol
        assert rel(g.matvec_t(xd).cpu().numpy(), O.matvec_t(o, x)) <= 1e-2 * tol
    g.free()
    # a single column longer than the limit is refused (every column here holds
    # more than 16 entries of at least 2 bytes)
    monkeypatch.setenv("HH_RUN_BYTES_MAX", "32")
    with pytest.raises(HHError) as ei:
        HMatrix(p.points, p.kernel, tol, p.eta, -1, 48)
    assert ei.value.status == 4


def test_autotune_keeps_products_and_picks_a_timed_setting():
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    rng = np.random.default_rng(12)
    P = rng.random((20000, 3))
    g = HMatrix(P, W.INV_R, 1e-6, 1.5, -1, 64)
    x = torch.from_numpy(rng.standard_normal(20000)).cuda()
    y0, yt0 = g.matvec(x), g.matvec_t(x)
    r = g.autotune()
    assert len(r["tried"]) == 9 and r["best"] in r["tried"]
    assert r["best"]["ms"] == min(t["ms"] for t in r["tried"])
    y1, yt1 = g.matvec(x), g.matvec_t(x)
    # other work units change only the summation order of the leaf rows
    assert float(torch.linalg.norm(y1 - y0) / torch.linalg.norm(y0)) <= 1e-13
    assert float(torch.linalg.norm(yt1 - yt0) / torch.linalg.norm(yt0)) <= 1e-13
    assert torch.equal(y1, g.matvec(x))
    # a handle built with the chosen sizes gives the tuned handle's products
    g2 = HMatrix(P, W.INV_R, 1e-6, 1.5, -1, 64, unit_bytes=r["best"]["unit_bytes"],
                 dot_task_elems=r["best"]["dot_task_elems"])
    assert torch.equal(g2.matvec(x), y1)
    g2.free()
    g.free()
