"""Writes tests/golden/oracle_3d_laplace_n131072.npz: the FP64 oracle's H_h
matrix of the 3D benchmark recipe at N = 2^17 (1/(4 pi r), points uniform in
[0,1]^3 from seed 303, leaf 256 so L = 3 and leaves of 256 points as in the
benchmark, eta 1.5, switching level L - 1 = 2, tol 1e-6, formats
{fp64, fp32, fp16, bf16}) and its products H^ x, H^^T x for x ~ N(0, 1)
(seed 1).

Only the oracle and the seeded input generators are called: every stored value
comes from oracle/hh_oracle.py. Building takes tens of minutes on a few cores,
which is why the GPU parity test reads the stored result instead of rebuilding
it. Run from the repository root:

    python tests/golden/make_oracle_reference.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W                      # noqa: E402
from oracle import hh_oracle as O          # noqa: E402

N = 1 << 17
OUT = os.path.join(ROOT, "tests", "golden", "oracle_3d_laplace_n131072.npz")


def main() -> None:
    p = W.cfg_3d_laplace(n=N, switch_level=-1)
    t0 = time.time()
    hm = O.build(p.points, O.Kernel(p.kernel, scale=p.scale), p.tol, p.eta, p.switch_level,
                 p.leaf_size, mask=p.mask, seed=p.seed)
    print(f"oracle build: {time.time() - t0:.1f} s, L = {hm.tree.L}, ell = {hm.ell}, "
          f"{len(hm.blocks)} blocks", flush=True)
    x = np.random.default_rng(1).standard_normal(N)
    y = O.matvec(hm, x)
    yt = O.matvec_t(hm, x)
    st = O.structure_arrays(hm)
    comp = [sb.comp for sb in hm.blocks]
    nan = float("nan")
    np.savez_compressed(
        OUT, n=N, L=hm.tree.L, ell=hm.ell, total2=hm.total2,
        level=st["level"], i=st["i"], j=st["j"], kind=st["kind"], lowrank=st["lowrank"],
        rank=st["rank"], fmt=st["fmt"],
        nb2=np.array([sb.nb2 for sb in hm.blocks]),
        tail=np.array([c.tail if c else nan for c in comp]),
        tail_prev=np.array([c.tail_prev if c else nan for c in comp]),
        thr=np.array([c.thr if c else nan for c in comp]),
        sketch=np.array([c.sketch if c else -1 for c in comp], dtype=np.int32),
        pmin=np.array([min(sb.blk.m, sb.blk.n) for sb in hm.blocks], dtype=np.int32),
        y=y, yt=yt)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
