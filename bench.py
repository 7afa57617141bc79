#!/usr/bin/env python3
"""Benchmark of the adaptive mixed-precision H_h mat-vec on one MI355X.

Workload (3D Laplace): N = 2^20 points uniform in [0,1]^3 (seed 303), kernel
1/(4 pi r), leaf 256 (L = 4), eta 1.5, switching level 3 (= L - 1), tol 1e-6,
formats {fp64, fp32, fp16, bf16} chosen per block by the paper's rule, one
right-hand side x ~ N(0, 1) in fp64. The same tree, partition and factors
stored uniformly in fp64 are timed beside it (built once; the adaptive handle
is derived from it, so both hold identical factors before rounding).

One step = one product y = H^ x (gather, inner products, leaf accumulation),
inputs resident in HBM. Prints one JSON line; `value` is adaptive matvec/s.
The roofline object covers the kernel with the largest share of the step
time, with its algorithmic bytes per launch over its mean event-timed
duration in the timed region. The CPU baseline is the FP64 oracle's own
product (Alg. 4) timed on the host on a smaller instance of the same recipe
(N = 16384, leaf 256, L = 2), run in a child process while the GPU builds,
and scaled to the headline by the ratio of stored entries.
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
CPU_SAMPLE_N = 16384


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


def cpu_worker(out_path: str, budget_s: float) -> None:
    """Build the oracle on the sample instance and time its product."""
    import numpy as np

    import workloads as W
    from oracle import hh_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    p = W.cfg_3d_laplace(n=CPU_SAMPLE_N)
    t0 = time.perf_counter()
    hm = O.build(p.points, O.Kernel(p.kernel, scale=p.scale), p.tol, p.eta, -1, p.leaf_size)
    t_build = time.perf_counter() - t0
    x = W.rhs(p.n, 1, np.random.default_rng(1))[:, 0]
    O.matvec(hm, x)
    reps, t0 = 0, time.perf_counter()
    while True:
        O.matvec(hm, x)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    entries = sum(sb.rank * (sb.blk.m + sb.blk.n) if sb.lowrank else sb.blk.m * sb.blk.n
                  for sb in hm.blocks)
    with open(out_path, "w") as f:
        json.dump({"seconds_per_matvec": el / reps, "reps": reps, "entries": entries,
                   "threads": threads, "build_seconds": t_build, "n": p.n, "L": hm.tree.L,
                   "ell": hm.ell}, f)


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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uniform", action="store_true", help="build the adaptive handle only")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-check", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--switch-level", action="store_true",
                    help="time the switching-level search (Alg. 2) at --n instead")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_budget)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: the H_h product here runs on a single MI355X "
              "(--gpus 1); multi-GPU runs are not part of this benchmark.", file=sys.stderr)
        return 2
    if args.switch_level:
        return switch_level_bench(args.n)

    # CPU baseline in a child process, overlapped with the GPU build
    worker = None
    wpath = None
    if not args.no_cpu_baseline:
        fd, wpath = tempfile.mkstemp(prefix="hh_cpu_", suffix=".json")
        os.close(fd)
        worker = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", wpath,
                                   "--cpu-budget", str(args.cpu_budget)], cwd=ROOT)

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
    if args.no_uniform:
        Ha = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale)
        H64 = None
    else:
        H64 = HMatrix(p.points, p.kernel, p.tol, p.eta, p.switch_level, p.leaf_size, scale=p.scale,
                      uniform_fp64=True)
        Ha = H64.derive(mask=0xF)
    t_build = time.perf_counter() - t0
    print(f"bench: built in {t_build:.1f} s", file=sys.stderr, flush=True)

    x = torch.from_numpy(W.rhs(p.n, args.nrhs, np.random.default_rng(1))).cuda()
    if args.nrhs == 1:
        x = x[:, 0].contiguous()

    def run(H):
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            H.matvec(x, out=y)
        torch.cuda.synchronize()
        ph = np.zeros(3)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, ms = H.matvec_timed(x, out=y)
            ph += ms
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return y, el, ph / args.steps

    ya, el_a, ph_a = run(Ha)
    sa = Ha.stats()
    res = {"adaptive": {"matvec_per_s": args.steps / el_a, "ms_per_step": 1000 * el_a / args.steps,
                        "phase_ms": [round(v, 4) for v in ph_a],
                        "phase_bytes": [int(v) for v in sa["phase_bytes"]],
                        "bytes_per_matvec": sa["matvec_bytes"],
                        "hbm_gbs": sa["matvec_bytes"] / (el_a / args.steps) / 1e9,
                        "blocks_by_format": sa["blocks_by_format"]}}
    if H64 is not None:
        y6, el_6, ph_6 = run(H64)
        s6 = H64.stats()
        res["uniform_fp64"] = {"matvec_per_s": args.steps / el_6,
                               "ms_per_step": 1000 * el_6 / args.steps,
                               "phase_ms": [round(v, 4) for v in ph_6],
                               "phase_bytes": [int(v) for v in s6["phase_bytes"]],
                               "bytes_per_matvec": s6["matvec_bytes"],
                               "hbm_gbs": s6["matvec_bytes"] / (el_6 / args.steps) / 1e9}
        res["speedup_vs_uniform_fp64"] = el_6 / el_a
        res["adaptive_vs_uniform_rel_diff"] = float(torch.linalg.norm(ya - y6) / torch.linalg.norm(y6))

    if args.copy_check:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    k = int(np.argmax(ph_a))
    if args.nrhs == 1:
        names = ["gather", "column inner products (dot1_kernel)",
                 "leaf accumulation (unit_kernel + finish_kernel)"]
        kernels = ["gather_kernel", "dot1_kernel", "accumulation"]
        achieved = sa["phase_bytes"][k] / (ph_a[k] / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": names[k], "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(kernels[k], p.n, args.nrhs)}
    else:
        # several right-hand sides: fp64 MFMA contractions, 2 R flops per stored
        # entry (phase V: V entries; phase U: U entries and dense entries)
        names = ["gather", "column inner products (dotm_kernel)", "leaf accumulation (accm_kernel)"]
        bl = Ha.blocks()
        lrm = bl["lowrank"].astype(bool)
        rk = bl["rank"].astype(np.float64)
        v_entries = float(np.sum((rk * (bl["col_end"] - bl["col_begin"]))[lrm]))
        u_entries = float(np.sum((rk * (bl["row_end"] - bl["row_begin"]))[lrm]))
        flops = [0.0, 2.0 * args.nrhs * v_entries, 2.0 * args.nrhs * (u_entries + sa["dense_entries"])]
        achieved = flops[k] / (ph_a[k] / 1e3) / 1e12
        roofline = {"bound": "mfma", "kernel": names[k], "achieved": round(achieved, 2),
                    "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFS, 4),
                    "traffic": None}

    cpu = None
    if worker is not None:
        try:
            worker.wait(timeout=900)
            with open(wpath) as f:
                w = json.load(f)
            headline_entries = sa["lowrank_entries"] + sa["dense_entries"]
            per_entry = w["seconds_per_matvec"] / w["entries"]
            cpu = {"value": 1.0 / (per_entry * headline_entries), "unit": "matvec/s",
                   "cores": w["threads"], "kind": "oracle",
                   "sample": (f"oracle Alg. 4 product on its own H_h of the same recipe at N={w['n']} "
                              f"(L={w['L']}, switch {w['ell']}): {w['seconds_per_matvec']*1e3:.2f} ms per "
                              f"product over {w['entries']} stored entries, {w['reps']} products; scaled "
                              f"to the {headline_entries} stored entries of the N={p.n} matrix")}
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
                                  f"{p.tol}, adaptive fp64/fp32/fp16/bf16, nrhs {args.nrhs}",
                      "n": p.n, "nrhs": args.nrhs, "build_seconds": round(t_build, 2),
                      "parallelism": "1 GPU"},
           "hbm_gbs": round(res["adaptive"]["hbm_gbs"], 1), "results": res,
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
