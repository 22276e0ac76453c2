"""Build libfmm.so (HIP, gfx950) in-tree: one hipcc compile per source file,
run in parallel, then one shared-library link."""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm.so")
SOURCES = ["api.hip", "sort.hip", "tree.hip", "walk.hip", "expansions.hip", "m2l.hip", "p2p.hip",
           "jerk.hip",
           "m2l_p01_06.hip", "m2l_p07_08.hip", "m2l_p09.hip", "m2l_p10.hip", "m2l_p11.hip",
           "m2l_p12.hip", "m2l_p13.hip", "m2l_p14.hip", "m2l_p15.hip", "m2l_p16.hip",
           "m2l32_p01_08.hip", "m2l32_p09_10.hip", "m2l32_p11.hip", "m2l32_p12.hip",
           "m2l32_p13.hip", "m2l32_p14.hip", "m2l32_p15.hip", "m2l32_p16.hip",
           "m2l_rot.hip", "m2lr_p01_08.hip", "m2lr_p09_11.hip", "m2lr_p12_13.hip",
           "m2lr_p14.hip", "m2lr_p15.hip", "m2lr_p16.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++20", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Wno-unused-function", "-I" + os.path.join(ROOT, "include"),
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-8000:]}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    # the highest-order M2L units take longest: start them first
    def cost(f):
        m = re.match(r"m2l(?:32|r)?_p(\d+)(?:_(\d+))?\.hip$", f)
        return int(m.group(2) or m.group(1)) if m else 0
    order = sorted(SOURCES, key=lambda f: -cost(f))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = dict(zip(order, ex.map(lambda s: _compile(s, verbose), order)))
    objs = [done[f] for f in SOURCES]
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
