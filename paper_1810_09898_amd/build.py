"""Build libsfcngb.so (HIP, gfx950) in-tree.

    python -m paper_1810_09898_amd.build

Every source under csrc/ is compiled with hipcc for gfx950 only and linked
into paper_1810_09898_amd/_lib/libsfcngb.so.  FP contraction is off so that
the FP64 membership test and the smoothing-length steps are rounded exactly
as written (explicit fma where the method wants one).  Packed FP32 ops are
disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libsfcngb.so")
SOURCES = ["sort.hip", "tree.hip", "group.hip", "search.hip", "abi.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src: str, obj: str, extra) -> None:
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    noisy = [ln for ln in (r.stderr or "").splitlines()
             if "warning" in ln and "packed-fp32-ops" not in ln]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")


def build(jobs: int = 8, extra=()) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        futs = []
        for s in SOURCES:
            obj = os.path.join(OUT_DIR, s.replace(".hip", ".o"))
            objs.append(obj)
            futs.append(ex.submit(_compile, os.path.join(CSRC, s), obj, list(extra)))
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build())
