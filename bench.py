#!/usr/bin/env python3
"""Benchmark of the adaptive mixed-precision H_h mat-vec on one MI355X.

Workload (3D Laplace): N = 2^20 points uniform in [0,1]^3 (seed 303), kernel
1/(4 pi r), leaf 256 (L = 4), eta 1.5, switching level 3 (= L - 1), tol 1e-6,
formats {fp64, fp32, fp16, bf16} chosen per block by the paper's rule, one
right-hand side x ~ N(0, 1) in fp64. The same tree, partition and factors
stored uniformly in fp64 are timed beside it (built once; the adaptive handle
is derived from it, so both hold identical factors before rounding).

One step = one product y = H^ x (gather, inner products, leaf accumulation),
inputs resident in HBM. The product is recorded once into a HIP graph; after
the warm-up replays, the K timed steps are K graph replays bracketed by device
synchronisations, each also bracketed by events on the replay stream (their
median is reported beside the wall-clock rate). `value` = adaptive products/s
over the K timed replays. The roofline object covers the kernel with the
largest share of the step: its algorithmic bytes per launch over its mean
duration, from HIP events the library records around each of its kernels on
the product's stream in K further eager products. The several-RHS rows
(16 and 256 right-hand sides on the same adaptive handle) are timed the same
way and carry an fp64-MFMA roofline each.

The CPU baseline is the FP64 oracle's own product (Alg. 4) on a bounded
sample of the same matrix, run in a child process while the GPU builds: the
oracle builds the headline's tree and partition, compresses a sample of its
blocks (every kind and level), times its product over those blocks and
scales the per-entry time to all stored entries of the GPU's matrix.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6        # dense fp64 MFMA


def measured_traffic(kernel: str, n: int, nrhs: int):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none for this workload or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2604_09147_amd", "csrc", "kernels_mv.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_mv_sha256") != sha or rec.get("n") != n or rec.get("nrhs") != nrhs:
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


def cpu_worker(out_path: str, budget_s: float, n: int) -> None:
    """The oracle's product (Alg. 4) on a bounded sample of the benchmark
    matrix. The oracle builds the tree and partition of the workload and
    compresses a few blocks of each (level, kind) group; each group's blocks,
    with their row and column ranges laid side by side in a short vector, form
    a small H matrix that O.matvec applies repeatedly (its O(length) gather and
    scatter, timed with no blocks, is subtracted). Level-2 blocks (16384^2, half
    a minute each for the oracle to generate and compress) are not sampled:
    their interaction-list rate is taken from the level-3 interaction list."""
    import dataclasses

    import numpy as np

    import workloads as W
    from oracle import hh_oracle as O
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=cores, user_api="blas")
    except Exception:
        pass
    p = W.cfg_3d_laplace(n=n)
    kern = O.Kernel(p.kernel, scale=p.scale)
    t0 = time.perf_counter()
    tree = O.build_tree(p.points, p.leaf_size)
    blocks = O.partition(tree, p.eta, p.switch_level)
    pt = p.points[tree.perm]
    rng = np.random.default_rng(7)
    groups = {}
    for q, b in enumerate(blocks):
        if b.level >= tree.L - 1:
            groups.setdefault((b.level, b.kind), []).append(q)
    stored = {}
    for key, qs in sorted(groups.items()):
        pick = rng.choice(qs, min(3 if key[0] < tree.L else 16, len(qs)), replace=False)
        sbs, off = [], 0
        for q in sorted(int(v) for v in pick):
            b = blocks[q]
            H = O.block_entries(pt, kern, None, b)
            # the block's rows and columns get their own slots of the short vector
            nb = dataclasses.replace(b, ib=off, ie=off + b.m, jb=off + b.m, je=off + b.m + b.n)
            off += b.m + b.n
            if b.kind == O.T_DIAG:
                sbs.append(O.StoredBlock(nb, q, False, D=H))
            else:
                c = O.compress(H, p.tol, p.seed, q)
                sbs.append(O.StoredBlock(nb, q, True, rank=c.rank, U=c.U, V=c.V))
        stored[key] = (sbs, off)
    t_prep = time.perf_counter() - t0

    def timed(sbs, length):
        sub = O.Tree(length, tree.d, tree.L, np.arange(length), None, None)
        hm = O.HMatrix(p.points, kern, sub, p.eta, p.switch_level, p.tol, 0xF, False, blocks=sbs)
        x = W.rhs(length, 1, np.random.default_rng(1))[:, 0]
        O.matvec(hm, x)
        reps, t1 = 0, time.perf_counter()
        while True:
            O.matvec(hm, x)
            reps += 1
            el = time.perf_counter() - t1
            if el >= budget_s / (2 * len(stored)) and reps >= 3:
                return el / reps, reps

    out = {"cores": cores, "prep_seconds": t_prep, "groups": []}
    for (level, kind), (sbs, length) in sorted(stored.items()):
        t, reps = timed(sbs, length)
        t_fix, _ = timed([], length)
        entries = sum(sb.rank * (sb.blk.m + sb.blk.n) if sb.lowrank else sb.blk.m * sb.blk.n
                      for sb in sbs)
        out["groups"].append({"level": level, "kind": kind, "blocks": len(sbs), "entries": entries,
                              "seconds": max(t - t_fix, 0.0), "reps": reps})
    x = W.rhs(p.n, 1, np.random.default_rng(1))[:, 0]
    hm0 = O.HMatrix(p.points, kern, tree, p.eta, p.switch_level, p.tol, 0xF, False, blocks=[])
    reps, t1 = 0, time.perf_counter()
    while reps < 5:
        O.matvec(hm0, x)
        reps += 1
    out["fixed_seconds"] = (time.perf_counter() - t1) / reps
    with open(out_path, "w") as f:
        json.dump(out, f)


def cpu_baseline(w: dict, bl: dict, n: int) -> dict:
    """Oracle products/s on the whole matrix: the O(N) gather / scatter of one
    product plus, per (level, kind) group, the sampled seconds per stored entry
    times the group's stored entries in the matrix (groups of coarser levels at
    the rate of the sampled interaction list of the coarsest sampled level)."""
    import numpy as np
    lr = bl["lowrank"].astype(bool)
    m = (bl["row_end"] - bl["row_begin"]).astype(np.float64)
    nn = (bl["col_end"] - bl["col_begin"]).astype(np.float64)
    ent = np.where(lr, bl["rank"] * (m + nn), m * nn)
    rate = {(g["level"], g["kind"]): g["seconds"] / max(g["entries"], 1) for g in w["groups"]}
    lmin = min(k[0] for k in rate)
    far = rate.get((lmin, 0), max(rate.values()))
    total = w["fixed_seconds"]
    for lev, kind in set(zip(bl["level"].tolist(), bl["kind"].tolist())):
        sel = (bl["level"] == lev) & (bl["kind"] == kind)
        total += rate.get((lev, kind), far) * float(np.sum(ent[sel]))
    parts = ", ".join(f"level {g['level']} kind {g['kind']}: {g['blocks']}" for g in w["groups"])
    return {"value": 1.0 / total, "unit": "matvec/s", "cores": w["cores"], "kind": "oracle",
            "sample": (f"oracle Alg. 4 product (O.matvec) over blocks of the N={n} matrix itself, "
                       f"compressed by the oracle ({parts} blocks per group), each group applied "
                       f"repeatedly on a vector holding just its rows and columns; seconds per stored "
                       f"entry of each group times the group's stored entries in the matrix (levels "
                       f"above {lmin} at the level-{lmin} interaction-list rate), plus the measured "
                       f"O(N) gather/scatter ({w['fixed_seconds'] * 1e3:.1f} ms); "
                       f"{w['cores']} BLAS threads")}


def graph_timing(H, x, y, steps: int, warmup: int):
    """Record one product into a HIP graph and replay it: (wall seconds of the
    `steps` timed replays, median replay ms from events on the replay stream)."""
    import torch
    H.reserve(1 if x.dim() == 1 else x.shape[1])
    H.matvec(x, out=y)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        H.matvec(x, out=y)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        graph.replay()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    del graph
    return wall, ms[len(ms) // 2]


def phase_timing(H, x, y, steps: int):
    """Mean [gather, inner products, leaf accumulation] ms over `steps` eager
    products with the library's per-kernel HIP events."""
    import numpy as np
    ph = np.zeros(3)
    for _ in range(steps):
        _, ms = H.matvec_timed(x, out=y)
        ph += ms
    return ph / steps


def switch_level_bench(n: int) -> int:
    """Time the switching-level search (Alg. 2: H_s, then H_h(ell) builds while
    the storage gain grows) on the 3D Laplace recipe at N = n, in the uniform
    fp64 and the mixed scheme; prints one JSON line of its own."""
    import torch

    import workloads as W
    from paper_2604_09147_amd import switch_level_search

    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    p = W.cfg_3d_laplace(n=n)
    out = {"metric": "switch_level_search_seconds", "unit": "s", "higher_is_better": False,
           "data": "synthetic",
           "config": {"workload": f"3D Laplace 1/(4 pi r), N={p.n} uniform in [0,1]^3, "
                                  f"leaf {p.leaf_size}, eta {p.eta}, tol {p.tol}"}}
    for name, uniform in (("uniform_fp64", True), ("adaptive", False)):
        print(f"bench: switching-level search, {name}, N={p.n}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = switch_level_search(p.points, p.kernel, p.tol, p.eta, p.leaf_size, scale=p.scale,
                                uniform_fp64=uniform)
        el = time.perf_counter() - t0
        walked = [l for l in range(r["L"] + 1) if not math.isnan(r["s2"][l])]
        out[name] = {"seconds": round(el, 2), "ell": r["ell"], "L": r["L"], "builds": len(walked),
                     "gain_words": {str(l): float(r["s1"][l] - r["s2"][l]) for l in walked},
                     "s1_words": [float(v) for v in r["s1"]]}
        print(f"bench: {name}: ell* = {r['ell']} in {el:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


def workload_bench(name: str, steps: int, warmup: int) -> int:
    """The other two configurations of the benchmark set, timed with graph
    replays like the headline: the 2D 1/r matrix (adaptive vs uniform fp64, 1
    and 64 right-hand sides) and the double-layer matrix (16 fp32 right-hand
    sides, the product with H and with H^T, as an autograd forward and
    backward pass would run them). q43: the 3D Laplace points at tol 1e-2,
    where the format rule picks the 8-bit q43 format for most blocks, with
    and without it in the mask (1 and 16 right-hand sides)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2604_09147_amd import HMatrix

    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    res = {}
    if name == "2d":
        p = W.cfg_2d_inv_r()
        t0 = time.perf_counter()
        H64 = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                      uniform_fp64=True)
        Ha = H64.derive(mask=0xF)
        t_build = time.perf_counter() - t0
        for H, tag in ((Ha, "adaptive"), (H64, "uniform_fp64")):
            H.autotune()
            st = H.stats()
            for R in (1, 64):
                shape = (p.n,) if R == 1 else (p.n, R)
                x = torch.from_numpy(W.rhs(p.n, R, np.random.default_rng(R))).reshape(shape).cuda()
                y = torch.empty_like(x)
                wall, med = graph_timing(H, x, y, steps, warmup)
                res[f"{tag}_nrhs{R}"] = {"ms_per_step": 1e3 * wall / steps,
                                         "graph_replay_ms_median": round(med, 4),
                                         "rhs_products_per_s": R * steps / wall,
                                         "hbm_gbs": st["matvec_bytes"] / (wall / steps) / 1e9}
                print(f"bench: {tag}, {R} RHS: {1e3 * wall / steps:.3f} ms", file=sys.stderr, flush=True)
        res["speedup_vs_uniform_fp64_nrhs1"] = (res["uniform_fp64_nrhs1"]["ms_per_step"] /
                                                res["adaptive_nrhs1"]["ms_per_step"])
        value, unit = res["adaptive_nrhs1"]["rhs_products_per_s"], "matvec/s"
        ms = res["adaptive_nrhs1"]["ms_per_step"]
        dtype = "f64"
        cfg = {"workload": f"2D 1/r, N={p.n} uniform in [0,1]^2, leaf {p.leaf_size}, eta {p.eta}, "
                           f"switch level {p.switch_level}, tol {p.tol}, adaptive fp64/fp32/fp16/bf16, "
                           "nrhs 1 (and 64)", "n": p.n, "nrhs": 1, "build_seconds": round(t_build, 2),
               "timing": "graph replays", "parallelism": "1 GPU"}
        blocks = Ha.stats()["blocks_by_format"]
        H64.free()
        Ha.free()
    elif name == "q43":
        p = W.cfg_3d_laplace()
        tol = 1e-2
        t0 = time.perf_counter()
        H64 = HMatrix(p.points, p.kernel, tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                      uniform_fp64=True)
        Hq = H64.derive(mask=0x2F)
        t_build = time.perf_counter() - t0
        Hf = H64.derive(mask=0xF)
        H64.free()
        for H, tag in ((Hq, "with_q43"), (Hf, "without_q43")):
            H.autotune()
            st = H.stats()
            for R in (1, 16):
                shape = (p.n,) if R == 1 else (p.n, R)
                x = torch.from_numpy(W.rhs(p.n, R, np.random.default_rng(R))).reshape(shape).cuda()
                y = torch.empty_like(x)
                wall, med = graph_timing(H, x, y, steps, warmup)
                res[f"{tag}_nrhs{R}"] = {"ms_per_step": 1e3 * wall / steps,
                                         "graph_replay_ms_median": round(med, 4),
                                         "rhs_products_per_s": R * steps / wall,
                                         "matvec_bytes": st["matvec_bytes"],
                                         "hbm_gbs": st["matvec_bytes"] / (wall / steps) / 1e9,
                                         "blocks_by_format": [int(v) for v in st["blocks_by_format"]]}
                print(f"bench: {tag}, {R} RHS: {1e3 * wall / steps:.3f} ms", file=sys.stderr, flush=True)
            x = torch.from_numpy(W.rhs(p.n, 1, np.random.default_rng(9))).cuda()
            res[f"{tag}_y"] = H.matvec(x)
        d = res.pop("with_q43_y") - res["without_q43_y"]
        res["rel_diff_with_vs_without_q43"] = float(d.norm() / res.pop("without_q43_y").norm())
        value, unit = res["with_q43_nrhs1"]["rhs_products_per_s"], "matvec/s"
        ms = res["with_q43_nrhs1"]["ms_per_step"]
        dtype = "q43/bf16 storage, fp32 + f64 arithmetic"
        cfg = {"workload": f"3D Laplace, N={p.n} uniform in [0,1]^3, leaf {p.leaf_size}, eta {p.eta}, "
                           f"switch level {p.switch_level}, tol {tol}, mask fp64/fp32/fp16/bf16/q43 "
                           "(and without q43), nrhs 1 (and 16)", "n": p.n, "nrhs": 1,
               "build_seconds": round(t_build, 2), "timing": "graph replays", "parallelism": "1 GPU"}
        blocks = Hq.stats()["blocks_by_format"]
        Hq.free()
        Hf.free()
    else:
        p = W.cfg_double_layer()
        t0 = time.perf_counter()
        H = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size,
                    normals=p.normals, io_dtype="f32")
        t_build = time.perf_counter() - t0
        H.autotune()
        st = H.stats()
        x = torch.from_numpy(W.rhs(p.n, 16, np.random.default_rng(5), np.float32)).cuda()
        for trans in (False, True):
            y = torch.empty_like(x)
            H.reserve(16)
            (H.matvec_t if trans else H.matvec)(x, out=y)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                (H.matvec_t if trans else H.matvec)(x, out=y)
            for _ in range(warmup):
                graph.replay()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(steps):
                graph.replay()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            tag = "transpose" if trans else "forward"
            res[tag] = {"ms_per_step": 1e3 * wall / steps, "rhs_products_per_s": 16 * steps / wall,
                        "hbm_gbs": st["matvec_bytes"] / (wall / steps) / 1e9}
            print(f"bench: double layer {tag}, 16 RHS: {1e3 * wall / steps:.3f} ms", file=sys.stderr,
                  flush=True)
            del graph
        value, unit = res["forward"]["rhs_products_per_s"], "RHS-products/s"
        ms = res["forward"]["ms_per_step"] + res["transpose"]["ms_per_step"]
        dtype = "f32 io, f64 accumulation"
        cfg = {"workload": f"double layer n_j.(p_i-p_j)/|p_i-p_j|^3, N={p.n} (half on the unit "
                           "sphere, half in the ball), leaf 256, eta 1.5, switch level 3, tol 1e-6, "
                           "16 fp32 RHS, H x then H^T g", "n": p.n, "nrhs": 16,
               "build_seconds": round(t_build, 2), "timing": "graph replays", "parallelism": "1 GPU"}
        blocks = st["blocks_by_format"]
        H.free()
    out = {"metric": f"H_h products, {name} workload", "value": round(value, 3), "unit": unit,
           "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded points, x ~ N(0,1))", "config": cfg,
           "blocks_by_format": [int(v) for v in blocks], "results": res}
    print(json.dumps(out), flush=True)
    return 0


def batched_bench(count: int, steps: int, warmup: int) -> int:
    """Independent Gaussian-kernel instances (N log-uniform in [2^10, 2^16], tol
    from {1e-4, 1e-6, 1e-8}, h ~ U[0.05, 0.3]), each built on the GPU with its
    own tree and precision rule, then multiplied together by hh_matvec_batch:
    one launch per phase over every handle, fp32 x and y."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2604_09147_amd import HMatrix, matvec_batch

    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    probs = W.cfg_batched()[:count]
    t0 = time.perf_counter()
    hs = []
    for i, p in enumerate(probs):
        t1 = time.perf_counter()
        hs.append(HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, h=p.h,
                          io_dtype="f32"))
        print(f"bench: instance {i}: N={p.n} tol={p.tol:.0e} h={p.h:.3f} built in "
              f"{time.perf_counter() - t1:.2f} s ({time.perf_counter() - t0:.1f} s in all)",
              file=sys.stderr, flush=True)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(4)
    xs = [torch.from_numpy(rng.standard_normal(h.n)).float().cuda() for h in hs]
    ys = [torch.empty_like(x) for x in xs]
    for _ in range(warmup):
        matvec_batch(hs, xs, ys)
    # one product of every instance alone, for the bitwise comparison
    singles = [h.matvec(x) for h, x in zip(hs, xs)]
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(ys, singles))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t1 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        matvec_batch(hs, xs, ys)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms = e0.elapsed_time(e1) / steps
    st = [h.stats() for h in hs]
    nbytes = float(sum(s["matvec_bytes"] for s in st))
    fmt = np.sum([s["blocks_by_format"] for s in st], axis=0)
    out = {"metric": "batched H_h instances: instance-products/s (one launch per phase)",
           "value": round(count * steps / wall, 1), "unit": "instance-products/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(1e3 * wall / steps, 4),
           "event_ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 io, f64 accumulation",
           "data": "synthetic (seeded points uniform in the unit cube, x ~ N(0,1))",
           "config": {"workload": f"{count} Gaussian-kernel instances exp(-r^2/h^2), N log-uniform "
                                  "in [2^10, 2^16], tol in {1e-4, 1e-6, 1e-8}, leaf 64, eta sqrt(3)",
                      "instances": count, "sum_n": int(sum(h.n for h in hs)),
                      "build_seconds": round(t_build, 2), "parallelism": "1 GPU"},
           "bytes_per_step": nbytes, "hbm_gbs": round(nbytes / (wall / steps) / 1e9, 1),
           "blocks_by_format": [int(v) for v in fmt], "batched_equals_single_products": same}
    print(json.dumps(out), flush=True)
    for h in hs:
        h.free()
    return 0 if same else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--multi-rhs", default="16,256",
                    help="right-hand-side counts timed on the adaptive handle after the "
                         "single-vector product ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default task sizes instead of the tuned ones")
    ap.add_argument("--no-uniform", action="store_true", help="build the adaptive handle only")
    ap.add_argument("--unit-bytes", type=int, default=0,
                    help="with --dot-task-elems: fixed task sizes for the adaptive handle "
                         "instead of the autotuner's (to profile a tuned configuration)")
    ap.add_argument("--dot-task-elems", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-check", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--switch-level", action="store_true",
                    help="time the switching-level search (Alg. 2) at --n instead")
    ap.add_argument("--batched", type=int, default=0, metavar="K",
                    help="time the batched workload instead: the first K of the 512 Gaussian "
                         "instances, one fp32 RHS each, in one launch per phase")
    ap.add_argument("--workload", default="headline", choices=["headline", "2d", "double_layer", "q43"],
                    help="2d: the 2D 1/r matrix (N=2^18, nrhs 1 and 64, adaptive vs uniform fp64); "
                         "double_layer: the double-layer matrix (N=2^19, 16 fp32 RHS, H and H^T); "
                         "q43: the 3D Laplace points at tol 1e-2 with and without q43 storage")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_budget, args.n)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: the H_h product here runs on a single MI355X "
              "(--gpus 1); multi-GPU runs are not part of this benchmark.", file=sys.stderr)
        return 2
    if args.switch_level:
        return switch_level_bench(args.n)
    if args.batched:
        return batched_bench(args.batched, args.steps, args.warmup)
    if args.workload != "headline":
        return workload_bench(args.workload, args.steps, args.warmup)
    multi = [int(v) for v in args.multi_rhs.split(",") if v.strip()]

    # CPU baseline in a child process, overlapped with the GPU build
    worker = None
    wpath = None
    if not args.no_cpu_baseline:
        fd, wpath = tempfile.mkstemp(prefix="hh_cpu_", suffix=".json")
        os.close(fd)
        worker = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", wpath,
                                   "--cpu-budget", str(args.cpu_budget), "--n", str(args.n)],
                                  cwd=ROOT)

    import numpy as np
    import torch

    import workloads as W
    from paper_2604_09147_amd import HMatrix

    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    p = W.cfg_3d_laplace(n=args.n)
    print(f"bench: building {p.name} N={p.n} leaf={p.leaf_size} eta={p.eta} "
          f"switch={p.switch_level} tol={p.tol}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    fixed_sizes = bool(args.unit_bytes and args.dot_task_elems)
    if fixed_sizes and not args.no_uniform:
        print("--unit-bytes / --dot-task-elems need --no-uniform", file=sys.stderr)
        return 2
    if args.no_uniform:
        Ha = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                     unit_bytes=args.unit_bytes, dot_task_elems=args.dot_task_elems)
        H64 = None
    else:
        H64 = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                      uniform_fp64=True)
        Ha = H64.derive(mask=0xF)
    t_build = time.perf_counter() - t0
    print(f"bench: built in {t_build:.1f} s", file=sys.stderr, flush=True)

    x = torch.from_numpy(W.rhs(p.n, 1, np.random.default_rng(1))[:, 0].copy()).cuda()

    tuned = {}

    def tune(H, name):
        if name == "adaptive" and fixed_sizes:
            tuned[name] = {"unit_bytes": args.unit_bytes, "dot_task_elems": args.dot_task_elems,
                           "ms": None}
            return
        if args.no_autotune:
            return
        r = H.autotune()
        tuned[name] = r["best"]
        print(f"bench: {name} task sizes {r['best']}", file=sys.stderr, flush=True)

    def run(H, xin):
        y = torch.empty_like(xin)
        wall, med = graph_timing(H, xin, y, args.steps, args.warmup)
        ph = phase_timing(H, xin, y, args.steps)
        torch.cuda.synchronize()
        return y.clone(), wall, med, ph

    tune(Ha, "adaptive")
    ya, el_a, med_a, ph_a = run(Ha, x)
    sa = Ha.stats()
    print(f"bench: adaptive {1e3 * el_a / args.steps:.3f} ms per product", file=sys.stderr, flush=True)
    res = {"adaptive": {"matvec_per_s": args.steps / el_a, "ms_per_step": 1000 * el_a / args.steps,
                        "graph_replay_ms_median": round(med_a, 4),
                        "phase_ms": [round(v, 4) for v in ph_a],
                        "phase_bytes": [int(v) for v in sa["phase_bytes"]],
                        "bytes_per_matvec": sa["matvec_bytes"],
                        "hbm_gbs": sa["matvec_bytes"] / (el_a / args.steps) / 1e9,
                        "blocks_by_format": sa["blocks_by_format"]}}
    if H64 is not None:
        tune(H64, "uniform_fp64")
        y6, el_6, med_6, ph_6 = run(H64, x)
        s6 = H64.stats()
        res["uniform_fp64"] = {"matvec_per_s": args.steps / el_6,
                               "ms_per_step": 1000 * el_6 / args.steps,
                               "graph_replay_ms_median": round(med_6, 4),
                               "phase_ms": [round(v, 4) for v in ph_6],
                               "phase_bytes": [int(v) for v in s6["phase_bytes"]],
                               "bytes_per_matvec": s6["matvec_bytes"],
                               "hbm_gbs": s6["matvec_bytes"] / (el_6 / args.steps) / 1e9}
        res["speedup_vs_uniform_fp64"] = el_6 / el_a
        res["adaptive_vs_uniform_rel_diff"] = float(torch.linalg.norm(ya - y6) / torch.linalg.norm(y6))
        # continuum storage of the same factors: per block t fraction bits, any t
        # in [7, 23] (continuum) or the byte-aligned t = 7, 15, 23 only
        for name, mode in (("continuum", 1), ("continuum_aligned", 2)):
            Hc = H64.derive(continuum=mode)
            tune(Hc, name)
            yc, el_c, med_c, ph_c = run(Hc, x)
            sc = Hc.stats()
            bc = Hc.blocks()
            tb = bc["frac_bits"][bc["format"] == 4]
            res[name] = {"matvec_per_s": args.steps / el_c, "ms_per_step": 1000 * el_c / args.steps,
                         "graph_replay_ms_median": round(med_c, 4),
                         "phase_ms": [round(v, 4) for v in ph_c],
                         "phase_bytes": [int(v) for v in sc["phase_bytes"]],
                         "bytes_per_matvec": sc["matvec_bytes"],
                         "hbm_gbs": sc["matvec_bytes"] / (el_c / args.steps) / 1e9,
                         "blocks_by_format": sc["blocks_by_format"],
                         "fraction_bits_histogram": {int(v): int(np.sum(tb == v)) for v in np.unique(tb)},
                         "speedup_vs_uniform_fp64": el_6 / el_c,
                         "rel_diff_vs_uniform_fp64": float(torch.linalg.norm(yc - y6) /
                                                           torch.linalg.norm(y6))}
            print(f"bench: {name} {1e3 * el_c / args.steps:.3f} ms per product", file=sys.stderr,
                  flush=True)
            Hc.free()
            del yc
            torch.cuda.empty_cache()
        H64.free()
        del y6
        torch.cuda.empty_cache()

    if args.copy_check:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    k = int(np.argmax(ph_a))
    names = ["gather", "column inner products (dot1_kernel)",
             "leaf accumulation (unit_kernel + finish_kernel)"]
    kernels = ["gather_kernel", "dot1_kernel", "accumulation"]
    achieved = sa["phase_bytes"][k] / (ph_a[k] / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": names[k], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kernels[k], p.n, 1)}

    # several right-hand sides on the adaptive handle: fp64 MFMA contractions,
    # 2 R flops per stored entry (phase V: V entries; phase U: U and dense entries)
    bl = Ha.blocks()
    if multi:
        lrm = bl["lowrank"].astype(bool)
        rk = bl["rank"].astype(np.float64)
        v_entries = float(np.sum((rk * (bl["col_end"] - bl["col_begin"]))[lrm]))
        u_entries = float(np.sum((rk * (bl["row_end"] - bl["row_begin"]))[lrm]))
        for R in multi:
            X = torch.from_numpy(W.rhs(p.n, R, np.random.default_rng(R))).cuda()
            Y, el_r, med_r, ph_r = run(Ha, X)
            col = int(np.random.default_rng(R + 1).integers(R))
            y1 = Ha.matvec(X[:, col].contiguous())
            flops = [0.0, 2.0 * R * v_entries, 2.0 * R * (u_entries + sa["dense_entries"])]
            kr = int(np.argmax(ph_r))
            ach = flops[kr] / (ph_r[kr] / 1e3) / 1e12
            total_tf = (flops[1] + flops[2]) / (el_r / args.steps) / 1e12
            res[f"adaptive_nrhs{R}"] = {
                "products_per_s": args.steps / el_r, "ms_per_step": 1000 * el_r / args.steps,
                "rhs_products_per_s": R * args.steps / el_r,
                "graph_replay_ms_median": round(med_r, 4),
                "phase_ms": [round(v, 4) for v in ph_r], "tflops_whole_product": round(total_tf, 2),
                "column_vs_single_rhs_rel_diff": float(torch.linalg.norm(Y[:, col] - y1) /
                                                       torch.linalg.norm(y1)),
                "roofline": {"bound": "mfma", "kernel": ["gather", "column inner products (dotm_kernel)",
                                                         "leaf accumulation (accm_kernel)"][kr],
                             "achieved": round(ach, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                             "frac": round(ach / FP64_PEAK_TFS, 4), "traffic": None}}
            print(f"bench: adaptive, {R} RHS: {1e3 * el_r / args.steps:.3f} ms per product",
                  file=sys.stderr, flush=True)
            del X, Y, y1
            torch.cuda.empty_cache()

    cpu = None
    if worker is not None:
        try:
            worker.wait(timeout=900)
            with open(wpath) as f:
                w = json.load(f)
            cpu = cpu_baseline(w, bl, p.n)
        except Exception as e:  # the baseline is reported, never required
            cpu = {"value": None, "unit": "matvec/s", "cores": None, "kind": "oracle",
                   "sample": f"unavailable: {e}"}
        finally:
            if wpath and os.path.exists(wpath):
                os.remove(wpath)

    value = res["adaptive"]["matvec_per_s"]
    out = {"metric": "H_h matvec/s + HBM GB/s, 3D 1/r N=2^20 tol 1e-6: adaptive vs uniform FP64",
           "value": round(value, 3), "unit": "matvec/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1000.0 / value, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded uniform points, x ~ N(0,1))",
           "config": {"workload": f"3D Laplace 1/(4 pi r), N={p.n} uniform in [0,1]^3, leaf "
                                  f"{p.leaf_size}, eta {p.eta}, switch level {p.switch_level}, tol "
                                  f"{p.tol}, adaptive fp64/fp32/fp16/bf16, nrhs 1",
                      "n": p.n, "nrhs": 1, "build_seconds": round(t_build, 2),
                      "timing": "graph replays", "parallelism": "1 GPU"},
           "hbm_gbs": round(res["adaptive"]["hbm_gbs"], 1), "results": res, "autotune": tuned,
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
