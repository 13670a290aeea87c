"""Build the HIP library ``libcmg.so`` in-tree for gfx950 with hipcc.

Every source is compiled to an object of its own (in parallel), then the
objects are linked into the shared library.

Flags: -ffp-contract=off keeps every floating-point expression in its
written order without fused multiply-add (results are reproducible bit for
bit); packed FP32 instructions are disabled; FP32 division and square root
are correctly rounded.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/kernels.hip", "csrc/fused.hip", "csrc/coarse.hip", "csrc/abfp.hip", "csrc/solver.hip"]
LIB = os.path.join(HERE, "libcmg.so")
OBJDIR = os.path.join(HERE, "_build")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return res.returncode, res.stdout + res.stderr


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, *FLAGS, *inc, "-c", os.path.join(HERE, src), "-o", obj])
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = [out for rc, out in results if rc != 0]
    if failed:
        sys.stderr.write("\n".join(failed))
        raise RuntimeError("hipcc failed to compile the HIP sources of libcmg.so")
    tmp = LIB + ".tmp"
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    if rc != 0:
        sys.stderr.write(out)
        raise RuntimeError("hipcc failed to link libcmg.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
