"""Build libgeosink.so in-tree with hipcc for gfx950.

    python -m paper_2211_00805_amd.build

Every translation unit is compiled in parallel into _build/ at the repository
root and linked into paper_2211_00805_amd/libgeosink.so.  Packed FP32 vector
instructions are disabled for device code (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgeosink.so")
SOURCES = ["kernels.hip", "euler.hip", "measure.hip", "accumulate.hip", "validate.hip", "knn.hip", "noalloc.hip", "frontier.hip", "coeffs.cpp", "graph.cpp", "plan.cpp", "abi.cpp"]
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-fopenmp",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> tuple[str, int, str]:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc(), *_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    return obj, p.returncode, msg


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, SOURCES))
    errors = [(o, m) for o, rc, m in results if rc != 0]
    for o, rc, m in results:
        if verbose and m.strip():
            print(m, file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(m for _, m in errors))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), *_flags(), "-shared", "-o", tmp, *[o for o, _, _ in results]]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
