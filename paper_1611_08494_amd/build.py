"""Builds libc3x.so for gfx950 in-tree (paper_1611_08494_amd/_build/).

Every HIP source is compiled with hipcc for gfx950 with FP contraction off
(decisions of the count and write passes must agree bit for bit; fused
operations are written out explicitly with fma) and packed-FP32 code
generation disabled. The binary128 fallback is plain C++ built with g++
against libquadmath.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libc3x.so")
HIP_SOURCES = ["c3x_common.hip", "c3x_sort.hip", "c3x_index.hip", "c3x_match.hip",
               "c3x_join.hip", "c3x_concentric.hip", "c3x_mutual.hip",
               "c3x_exact.hip", "c3x_frames.hip"]
ARCH = os.environ.get("C3X_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        objs.append(obj)
        jobs.append([hipcc, *HIPCC_FLAGS, "-c", path, "-o", obj])
    qobj = os.path.join(OUT, "exact128.o")
    jobs.append(["g++", "-O2", "-std=gnu++17", "-fPIC", "-c", os.path.join(CSRC, "exact128.cpp"),
                 "-o", qobj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, qobj, "-lquadmath",
          "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
