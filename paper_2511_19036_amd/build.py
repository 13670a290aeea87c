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
# A second build whose host code runs under AddressSanitizer and
# UndefinedBehaviorSanitizer (the device code is built as usual), for the
# host-side tests of the C ABI; it needs the sanitizer runtime preloaded.
SAN_LIB = os.path.join(HERE, "_build_san", "libcmg_sanitized.so")
SAN_OBJDIR = os.path.join(HERE, "_build_san")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all", "-g"]

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


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime of the ROCm compiler (to preload
    into a process that loads the sanitized library)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    res = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the ROCm compiler's AddressSanitizer runtime was not found")
    return path


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link libcmg.so (or, with sanitize, the
    host-sanitized library at SAN_LIB).  Returns the library path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir, lib = (SAN_OBJDIR, SAN_LIB) if sanitize else (OBJDIR, LIB)
    extra = SAN_FLAGS if sanitize else []
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, *FLAGS, *extra, *inc, "-c", os.path.join(HERE, src), "-o", obj])
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = [out for rc, out in results if rc != 0]
    if failed:
        sys.stderr.write("\n".join(failed))
        raise RuntimeError("hipcc failed to compile the HIP sources of libcmg.so")
    tmp = lib + ".tmp"
    link = ["-shared-libasan", *SAN_FLAGS] if sanitize else []
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *link, "-o", tmp], verbose)
    if rc != 0:
        sys.stderr.write(out)
        raise RuntimeError("hipcc failed to link " + os.path.basename(lib))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
