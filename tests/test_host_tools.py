"""CPU tests of the host-side tooling around the product: the benchmark's
one-GPU refusal, its lookup of the committed HBM counter summary, the loud
failure of the binding when the library has not been built (there is no CPU
fallback path), and the binding's argument checks, which run before any
device pointer reaches the library."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line for a refused run


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_measured_traffic_matches_summary_only_for_its_workload():
    bench = _bench()
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2604_09147_amd", "csrc", "kernels_mv.hip"), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == rec["kernels_mv_sha256"]
    n, nrhs = rec["n"], rec["nrhs"]
    for kern, ent in rec["kernels"].items():
        got = bench.measured_traffic(kern, n, nrhs)
        # a summary taken before the kernel source last changed is not used
        assert got == (ent["bytes_per_launch"] if current else None), kern
        assert bench.measured_traffic(kern, n // 2, nrhs) is None
        assert bench.measured_traffic(kern, n, nrhs + 15) is None
    assert bench.measured_traffic("no_such_kernel", n, nrhs) is None


def test_measured_traffic_rejects_a_stale_source_hash(tmp_path, monkeypatch):
    bench = _bench()
    # a copy of the tree layout with the summary of one kernel and a source
    # whose hash differs from the recorded one
    (tmp_path / "profiles").mkdir()
    src_dir = tmp_path / "paper_2604_09147_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (src_dir / "kernels_mv.hip").write_bytes(b"// kernel source\n")
    good = hashlib.sha256(b"// kernel source\n").hexdigest()
    rec = {"n": 64, "nrhs": 1, "kernels_mv_sha256": good,
           "kernels": {"k": {"bytes_per_launch": 1234}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k", 64, 1) == 1234
    (src_dir / "kernels_mv.hip").write_bytes(b"// kernel source, changed\n")
    assert bench.measured_traffic("k", 64, 1) is None
    (tmp_path / "profiles" / "traffic.json").write_text("{not json")
    assert bench.measured_traffic("k", 64, 1) is None


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    from paper_2604_09147_amd import hh
    monkeypatch.setattr(hh, "LIB_PATH", str(tmp_path / "libhhmat.so"))
    monkeypatch.setattr(hh, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        hh.lib()


def _fake_handle(n, io="f64"):
    # an HMatrix shell with no native handle: enough for the argument checks,
    # which run before any library call
    from paper_2604_09147_amd.hh import HMatrix
    m = HMatrix.__new__(HMatrix)
    m._h = None
    m.n = n
    m.io_dtype = io
    return m


def test_product_arguments_checked_before_the_library():
    import torch
    from paper_2604_09147_amd import matvec_batch
    a, b = _fake_handle(10), _fake_handle(12)
    with pytest.raises(ValueError, match="device tensor"):
        a.matvec(torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="one x"):
        matvec_batch([a, b], [torch.zeros(10, dtype=torch.float64)])
    with pytest.raises(ValueError, match="one x"):
        matvec_batch([], [])
    with pytest.raises(ValueError, match="device tensor"):
        matvec_batch([a, b], [torch.zeros(10, dtype=torch.float64), torch.zeros(12, dtype=torch.float64)])
