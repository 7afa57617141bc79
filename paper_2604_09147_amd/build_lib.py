"""Compile the HIP sources into lib/libhhmat.so (gfx950) with hipcc.

Used by ``__graft_entry__.build()`` and runnable as a script. Every call
recompiles; objects go to a temporary directory, the library into ``lib/``."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libhhmat.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

SOURCES = ["plan.cpp", "capi.cpp", "solve.cpp", "build.hip", "kernels_build.hip", "kernels_mv.hip"]

COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{os.path.join(HERE, '..', 'include')}",
          f"-I{ROCM}/include", "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src: str, obj: str) -> None:
    path = os.path.join(SRC, src)
    cmd = [os.path.join(ROCM, "bin", "hipcc")] + COMMON
    if src.endswith(".hip") or src in ("capi.cpp", "solve.cpp"):
        cmd += ["-x", "hip"] + DEVICE
    else:
        cmd += ["-x", "c++"]
    if src == "plan.cpp":
        cmd += ["-ffp-contract=off"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = tempfile.mkdtemp(prefix="hhmat_build_")
    try:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
            list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
        out_tmp = LIB + ".tmp"
        cmd = [os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-shared", "-fPIC",
               "-o", out_tmp] + objs + [f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas",
                                        f"-Wl,-rpath,{ROCM}/lib"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB)
        if verbose:
            print(f"built {LIB}")
        return LIB
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
