"""Compile the HIP library libdeg.so for gfx950 (in-tree, parallel per source).

    python -m paper_2307_10479_amd.build_lib
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = PKG / "_build"
LIB = PKG / "libdeg.so"
SOURCES = ["search.hip", "search_f32.hip", "search_bf16.hip", "search_fp8.hip", "util.hip",
           "knn.hip", "mlp.hip", "build.hip", "graph_check.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-I" + str(ROOT / "include"),
         "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


# host-side flags per source: the construction's host edits compute FP32 distances
# with fused multiply-adds (hardware FMA instead of a libm call per term; every
# x86 host of an MI355X node has FMA and AVX2)
HOST_FLAGS = {"build.hip": ["-Xarch_host", "-mavx2", "-Xarch_host", "-mfma"]}


def _compile(src: str) -> Path:
    obj = BUILD / (src + ".o")
    dep = [CSRC / src] + sorted(CSRC.glob("*.h")) + [ROOT / "include" / "deg.h"]
    if obj.exists() and all(obj.stat().st_mtime >= d.stat().st_mtime for d in dep):
        return obj
    cmd = ["hipcc"] + FLAGS + HOST_FLAGS.get(src, []) + ["-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(force: bool = False, jobs: int | None = None) -> Path:
    BUILD.mkdir(exist_ok=True)
    if force:
        for o in BUILD.glob("*.o"):
            o.unlink()
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", str(tmp)] + [str(o) for o in objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    print(LIB)
