"""Benchmark: compact FMG on one MI355X, DoF/s to discretisation accuracy.

Workload (default): 3-D Poisson, 7-point finite differences, 1025^3 nodes
(1023^3 = 1.07e9 interior DoF), f = 3 pi^2 sin sin sin + 1e-4 U[-1, 1)
(counter-hashed, seed 3), compact FMG with N = 2 IR iterations per level,
V(2,2) red-black Gauss-Seidel in FP32, FP64 residual and coarsest solve,
BFP sections with blocks of 64 and 16-bit finest widths.  One step is one
full FMG solve with f already resident in HBM.

Prints ONE JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
# VALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD
# every 4 cycles (16 lanes per SIMD), 2.4 GHz.
VALU_PEAK = 256 * 4 / 4 * 2.4e9  # wave instructions per second
CALIB_BYTES = 1 << 30  # size of the calibration copy of the --pmc-pass mode
# the diffusion pass uses a size no other copy of that run has (building the
# coefficients copies 1 GiB arrays)
CALIB_BYTES_DIFF = 3 << 29


def log(msg):
    print(msg, file=sys.stderr, flush=True)


FUSED_SOURCES = ("fused.hip", "plane.h", "device.h")
# every kernel and the schedule that launches them (the diffusion workload
# runs the per-operation kernels)
ALL_SOURCES = ("kernels.hip", "coarse.hip", "fused.hip", "plane.h", "device.h", "launch.h", "solver.hip")


def kernel_source_digest(names=FUSED_SOURCES):
    """SHA-256 of kernel sources (by default fused.hip and the device headers
    it includes) with comments and blank lines removed, to tell whether
    stored counter readings still describe the kernels being run."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2511_19036_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()


def _stored_column(fname, kernel, col):
    """Column `col` of `kernel`'s row in a committed counter summary under
    profiles/, or None when the summary is missing or the kernel sources
    changed since its counters were taken."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    digest, per_launch = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("| `") and line.count("|") > col + 1:
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                try:
                    per_launch[cells[0].strip("`")] = float(cells[col])
                except ValueError:
                    pass
    if digest != kernel_source_digest():
        return None
    return per_launch.get(kernel)


def stored_diffusion_hbm():
    """The measured HBM rate of the compact 513^3 diffusion solve (GB/s, from
    the committed summary of its counter passes), or None when the summary
    is missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_diffusion3d_513x8.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            key, sep, val = line.partition(":")
            if sep and key in ("measured_gbs", "source_sha256_all"):
                vals[key] = val.strip()
    if vals.get("source_sha256_all") != kernel_source_digest(ALL_SOURCES) or "measured_gbs" not in vals:
        return None
    return float(vals["measured_gbs"])


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    against a copy of known size) from the committed counter summary."""
    return _stored_column("hbm_traffic_fused_kernels_poisson3d_1025.md", kernel, 5)


def stored_valu(kernel):
    """VALU wave instructions per launch of `kernel` (SQ_INSTS_VALU) from the
    committed counter summary."""
    return _stored_column("valu_issue_fused_kernels_poisson3d_1025.md", kernel, 2)


def model_bytes_per_dof(kernel, bits, block):
    """Algorithmic HBM bytes per interior DoF of one launch of a fused level
    kernel on the finest level (every section at the finest width `bits`,
    one int16 exponent per block): beta = bits / 8 + 2 / block bytes per
    stored value; the coarse level has 1/8 of the values.
      up sweep:     g, y' read; u' read and written; coarse y' and FP32 z read
      down sweep:   g read, y' written
      restriction:  g, y' read, coarse g written
      IR residual:  u' and coarse u' read, FP64 u two levels down read (the
                    coarse solution is rebuilt in the kernel), FP64 f read,
                    g written
      final decode: u' read, coarse FP64 u read, FP64 u written"""
    beta = bits / 8.0 + 2.0 / block
    name = kernel.partition("<")[0]
    table = {"k_up_smooth": 4 * beta + (beta + 4.0) / 8.0, "k_down_smooth": 2 * beta,
             "k_resid_restrict": 2 * beta + beta / 8.0, "k_ir_residual": 2 * beta + beta / 8.0 + 8.0 / 64.0 + 8.0,
             "k_decode_full": beta + 1.0 + 8.0}
    return table[name]


def _by_kernel(rows):
    """Per-level timing rows ("name@l") summed per kernel name."""
    acc = {}
    for r in rows:
        name = r["kernel"].partition("@")[0]
        a = acc.setdefault(name, dict(kernel=name, launches=0, ms=0.0, bytes=0.0))
        a["launches"] += r["launches"]
        a["ms"] += r["ms"]
        a["bytes"] += r["bytes"]
    return sorted(acc.values(), key=lambda r: -r["ms"])


def _family(kernel_name):
    """The library's timing name of a fused level kernel from a profiler
    name ("void cmg::k_up_smooth<4, 32, 768, 6, false, 16>(...)" ->
    "k_up_smooth<4>"), with its container template argument; (None, None)
    for other kernels."""
    import re
    m = re.search(r"cmg::(k_up_smooth|k_down_smooth|k_ir_residual|k_resid_restrict|k_decode_full)<([^>]*)>",
                  kernel_name)
    if not m:
        return None, None
    name, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
    if name in ("k_up_smooth", "k_down_smooth"):
        name = f"{name}<{args[0]}>"
    elif name == "k_decode_full" and args[2] == "true":
        name = "k_decode_level"
    # the container is the last integer argument (the IR residual and the
    # decode end with a flag: whether they rebuild the coarse solution)
    return name, int([a for a in args if a not in ("true", "false")][-1])


def summarize_counters(d, L, bits, block=64):
    """Markdown rows of the counter passes in directory d (rocprofv3 csv
    output of bench.py --pmc-pass: fetch_, write_ and valu_
    counter_collection.csv): per fused kernel family, HBM bytes per launch
    over the measured solve (after the calibration copy), FETCH_SIZE and
    WRITE_SIZE scaled by what they read for the runtime's copy of
    CALIB_BYTES; and the same for the launches on the finest level (the
    instantiation with the finest level's container), beside the per-DoF
    model's bytes; then the VALU/SALU/LDS instruction counts per launch."""
    import csv
    import collections

    def load(name):
        path = os.path.join(d, f"{name}_counter_collection.csv")
        return list(csv.DictReader(open(path))) if os.path.exists(path) else []

    def measured(rows):
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        calib = max(copies, key=lambda r: float(r["Counter_Value"]))
        return calib, [r for r in rows if int(r["Dispatch_Id"]) > int(calib["Dispatch_Id"])]

    cbits = 8 if bits <= 8 else 12 if bits <= 12 else 16 if bits <= 16 else 32
    dofs = ((1 << L) - 1) ** 3
    out = []
    per = {}
    for pas in ("fetch", "write"):
        rows = load(pas)
        calib, rows = measured(rows)
        scale = CALIB_BYTES / (float(calib["Counter_Value"]) * 1024.0)
        acc = collections.defaultdict(lambda: [0, 0.0])
        for r in rows:
            fam, cb = _family(r["Kernel_Name"])
            if fam is None:
                continue
            for key in ([fam] + ([f"{fam}@{L}"] if cb == cbits and fam != "k_decode_level" else [])):
                acc[key][0] += 1
                acc[key][1] += float(r["Counter_Value"])
        per[pas] = (scale, float(calib["Counter_Value"]), acc)
    fs, fcal, fa = per["fetch"]
    ws, wcal, wa = per["write"]
    out.append(f"Calibration: the runtime's device-to-device copy of {CALIB_BYTES} bytes reads FETCH_SIZE = "
               f"{fcal:.1f} KiB and WRITE_SIZE = {wcal:.1f} KiB, so FETCH_SIZE is scaled by {fs:.4f} and "
               f"WRITE_SIZE by {ws:.4f} to give bytes.")
    out.append("")
    out.append("| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | model bytes | HBM bytes (calibrated) "
               "| HBM / model |")
    out.append("|---|---:|---:|---:|---:|---:|---:|")
    for key in sorted(fa, key=lambda k: ("@" in k, k)):
        n, fkib = fa[key]
        wkib = wa[key][1] if key in wa else 0.0
        fk, wk = fkib / n, wkib / n
        hbm = fk * 1024.0 * fs + wk * 1024.0 * ws
        if "@" in key:
            model = model_bytes_per_dof(key.partition("@")[0], bits, block) * dofs
            out.append(f"| `{key}` | {n} | {fk:.1f} | {wk:.1f} | {model:.4e} | {hbm:.4e} | {hbm / model:.2f} |")
        else:
            out.append(f"| `{key}` | {n} | {fk:.1f} | {wk:.1f} | - | {hbm:.4e} | - |")
    vrows = load("valu")
    if vrows:
        vrows = measured(vrows)[1] if any("copyBuffer" in r["Kernel_Name"] for r in vrows) else vrows
        ids = sorted({int(r["Dispatch_Id"]) for r in vrows})
        half = ids[len(ids) // 2]  # the second (measured) solve of the pass
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        cnt = collections.defaultdict(set)
        for r in vrows:
            if int(r["Dispatch_Id"]) < half:
                continue
            fam, cb = _family(r["Kernel_Name"])
            if fam is None:
                continue
            for key in ([fam] + ([f"{fam}@{L}"] if cb == cbits and fam != "k_decode_level" else [])):
                acc[key][r["Counter_Name"]] += float(r["Counter_Value"])
                cnt[key].add(int(r["Dispatch_Id"]))
        out.append("")
        out.append("| kernel | launches | SQ_INSTS_VALU | SQ_INSTS_SALU | SQ_INSTS_LDS | SQ_WAVES |")
        out.append("|---|---:|---:|---:|---:|---:|")
        for key in sorted(acc, key=lambda k: ("@" in k, k)):
            n = len(cnt[key])
            c = acc[key]
            out.append(f"| `{key}` | {n} | {c['SQ_INSTS_VALU'] / n:.4e} | {c['SQ_INSTS_SALU'] / n:.4e} | "
                       f"{c['SQ_INSTS_LDS'] / n:.4e} | {c['SQ_WAVES'] / n:.4e} |")
    return "\n".join(out)


STALL_COUNTERS = (("sa", ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                           "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS")),
                  ("sb", ("SQ_ACTIVE_INST_SCA", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_MISC",
                          "SQ_INSTS_SALU", "SQ_INSTS_VALU")))


def summarize_stalls(d, L, bits):
    """Markdown rows of the two SQ counter passes in directory d (rocprofv3
    csv output of bench.py --pmc-pass, passes sa_ and sb_ with the counters
    of STALL_COUNTERS): for the fused kernels on the finest level (the
    instantiation with the finest level's container), over the launches of
    the second (measured) solve, where the waves' cycles go as fractions of
    SQ_WAVE_CYCLES (summed over waves): issuing an instruction (active),
    waiting on a memory, LDS or barrier counter (wait_any), waiting for an
    issue slot (wait_inst), and the VALU, scalar and LDS instructions and
    the LDS bank-conflict cycles among them."""
    import csv
    import collections
    cbits = 8 if bits <= 8 else 12 if bits <= 12 else 16 if bits <= 16 else 32
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    launches = collections.defaultdict(set)
    for pas, _ in STALL_COUNTERS:
        path = os.path.join(d, f"{pas}_counter_collection.csv")
        if not os.path.exists(path):
            continue
        rows = list(csv.DictReader(open(path)))
        ids = sorted({int(r["Dispatch_Id"]) for r in rows})
        half = ids[len(ids) // 2]  # the second (measured) solve of the pass
        for r in rows:
            fam, cb = _family(r["Kernel_Name"])
            if fam is None or int(r["Dispatch_Id"]) < half or cb != cbits or fam == "k_decode_level":
                continue
            key = f"{fam}@{L}"
            acc[key][r["Counter_Name"]] += float(r["Counter_Value"])
            if pas == "sa":
                launches[key].add(int(r["Dispatch_Id"]))
    out = ["| kernel | launches | wave cycles per launch | active | wait_any | wait_inst | VALU | scalar | LDS "
           "| LDS bank conflict |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for key in sorted(acc):
        c = acc[key]
        n = max(len(launches[key]), 1)
        wc = c.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        frac = [c.get(name, 0.0) / wc for name in ("SQ_ACTIVE_INST_ANY", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                                                    "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA",
                                                    "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT")]
        out.append(f"| `{key}` | {n} | {c.get('SQ_WAVE_CYCLES', 0.0) / n:.4e} | "
                   + " | ".join(f"{x:.3f}" for x in frac) + " |")
    return "\n".join(out)


def discretisation_check(u, L, dim=3):
    """Errors of u against the closed-form discrete solution of the sine part.

    For f = d pi^2 prod sin(pi x) the 7-point solution is c_h u* with
    c_h = ((pi h / 2) / sin(pi h / 2))^2; the 1e-4 noise moves the discrete
    solution by ~1e-10 relative, far below the discretisation error.
    """
    import torch
    h = 2.0 ** -L
    N = (1 << L) + 1
    x = torch.arange(N, dtype=torch.float64, device=u.device) * h
    s = torch.sin(math.pi * x)
    s[0] = 0.0
    s[-1] = 0.0
    ch = ((math.pi * h / 2) / math.sin(math.pi * h / 2)) ** 2
    err2 = dev2 = disc2 = 0.0
    for k in range(N):                      # plane by plane: no full-size temporaries
        us = s[k] * (s[:, None] * s[None, :])
        uk = u[k]
        err2 += float(((uk - us) ** 2).sum())
        dev2 += float(((uk - ch * us) ** 2).sum())
        disc2 += float((((ch - 1.0) * us) ** 2).sum())
    return math.sqrt(err2 / disc2), math.sqrt(dev2 / disc2)


_ORACLE_CHILD = """
import sys, time
sys.path.insert(0, {root!r})
import synthetic
from oracle import compact as oc
f = synthetic.hash_noise_rhs(3, {L}, amp=1e-4, seed=3)
cfg = oc.Config(dim=3, L={L}, smoother="rbgs", omega=1.0, block=64, bits_u={b}, bits_r={b}, bits_y={b})
print("start", time.time(), flush=True)
sys.stdin.readline()
t0 = time.time()
oc.fmg_solve(f, cfg)
print("solve", t0, time.time(), flush=True)
"""


def host_info():
    """Host cores and CPU model of the machine the benchmark runs on."""
    model = None
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return dict(nproc=os.cpu_count(), lscpu_model=model)


def cpu_baseline(L_sample: int, bits: int, procs: int):
    """The oracle (numpy, as it stands: single-threaded) on the same problem
    at a smaller grid: one solve on one host thread, then `procs` independent
    solves at once in child processes (one thread each) for the rate of all
    the host cores the GPU's share allows."""
    import subprocess
    code = _ORACLE_CHILD.format(root=ROOT, L=L_sample, b=bits)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    dofs = ((1 << L_sample) - 1) ** 3

    def run(n):
        ch = [subprocess.Popen([sys.executable, "-c", code], stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                               text=True, env=env) for _ in range(n)]
        for c in ch:  # every child has built its input; then all solve at once
            c.stdout.readline()
        for c in ch:
            c.stdin.write("go\n")
            c.stdin.flush()
        spans = []
        for c in ch:
            out, _ = c.communicate(timeout=600)
            if c.returncode != 0:
                raise RuntimeError("oracle child process failed")
            t0, t1 = [float(v) for v in out.split()[1:3]]
            spans.append((t0, t1))
        return min(a for a, _ in spans), max(b for _, b in spans)

    a, b = run(1)
    t1 = b - a
    a, b = run(procs)
    tp = b - a
    info = host_info()
    return dict(value=procs * dofs / tp, unit="DoF/s", cores=procs, kind="oracle",
                sample=f"the same problem and solver settings at {(1 << L_sample) + 1}^3 ({dofs} DoF): {procs} "
                       f"independent FMG solves at once, one per host core, {tp:.1f} s wall",
                single_thread=dict(value=dofs / t1, unit="DoF/s", cores=1,
                                   sample=f"one FMG solve at {(1 << L_sample) + 1}^3, {t1:.1f} s on one thread"),
                nproc=info["nproc"], lscpu_model=info["lscpu_model"],
                note="the oracle is plain numpy (no threading of its own); the all-core rate runs one solve per "
                     "core, capped at the host share of one GPU")


def _time_solves(s, f, reps):
    import torch
    u = torch.empty_like(f)
    s.solve(f, u)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        s.solve(f, u)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, u


def codec_rates(x, bits, reps=3):
    """Adaptive-exponent BFP (Sec. 6.1.3) encode and decode of the solution
    vector: one pass each; algorithmic bytes = the float64 values plus the
    codes (the block list and the look-back words are negligible)."""
    import torch

    from paper_2511_19036_amd import abfp_decode, abfp_encode, abfp_workspace
    n = x.numel()
    log(f"[bench] adaptive-exponent codec on the {n}-value solution, {bits} bits")
    ws = abfp_workspace(n)
    enc = abfp_encode(x, bits, workspace=ws)
    dec = abfp_decode(*enc, n, bits)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        enc = abfp_encode(x, bits, workspace=ws)
    e[1].record()
    e[2].record()
    for _ in range(reps):
        dec = abfp_decode(*enc, n, bits)
    e[3].record()
    torch.cuda.synchronize()
    t_enc, t_dec = e[0].elapsed_time(e[1]) / reps, e[2].elapsed_time(e[3]) / reps
    nb = int(enc[3].item())
    cbytes = enc[0].numel()
    moved = 8.0 * n + cbytes
    err = float(torch.max(torch.abs(dec - x)))
    amax = float(torch.max(torch.abs(x)))
    return dict(n=n, bits=bits, nblocks=nb, encode_ms=t_enc, encode_gbs=moved / (t_enc * 1e-3) / 1e9,
                encode_frac=moved / (t_enc * 1e-3) / HBM_PEAK, decode_ms=t_dec,
                decode_gbs=moved / (t_dec * 1e-3) / 1e9, decode_frac=moved / (t_dec * 1e-3) / HBM_PEAK,
                storage_bytes=cbytes + 10 * max(nb, 0), fixed_block64_bytes=cbytes + 2 * ((n + 63) // 64),
                max_abs_err=err, max_abs=amax)


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _converged(dim, L, f, iters=30, **kw):
    """A float64 solve run to stagnation (plain storage, float64 V-cycles,
    `iters` extra IR iterations on the finest level): the reference the
    other solves' errors are stated against."""
    from paper_2511_19036_amd import Solver
    with Solver(dim, L, batch=f.shape[0], storage="plain", vcycle_prec="fp64", final_iters=iters, **kw) as s:
        return s.solve(f)


def _coarsen_cells(k):
    n = k.shape[0] // 2
    return k.reshape(n, 2, n, 2, n, 2).mean(dim=(1, 3, 5)).contiguous()


def _richardson(uh, u2h):
    """Relative discretisation-error estimate of the second-order scheme
    from solutions on h and 2h at coincident nodes: |u_h - u_2h| / 3."""
    import torch
    c = uh[::2, ::2, ::2]
    return float(torch.linalg.vector_norm(c - u2h) / 3.0 / torch.linalg.vector_norm(c))


def _timed(fn, reps):
    import torch
    out = fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def other_workloads():
    """Solve times of the other workloads (same library, same GPU), each
    with its error against a converged float64 solve of the same system."""
    import torch

    import synthetic
    from paper_2511_19036_amd import Solver
    W = synthetic.WORKLOADS
    out = {}
    log("[bench] other workloads: 2-D 129^2, 3-D 257^3, diffusion 129^3 and 513^3 x 8")
    # config 1: 2-D, weighted Jacobi, compact against plain float64 FMG
    f = torch.from_numpy(synthetic.gaussian_noise_rhs(2, 7, 1e-3, 0)).cuda()[None].contiguous()
    ref = _converged(2, 7, f, smoother="wjacobi", omega=0.8)
    with Solver(2, 7, smoother="wjacobi", omega=0.8, bfp_block=32, bits=16) as s:
        ms, u = _timed(lambda: s.solve(f), 20)
    with Solver(2, 7, smoother="wjacobi", omega=0.8, storage="plain", vcycle_prec="fp64") as s:
        pms, up = _timed(lambda: s.solve(f), 20)
    h = 2.0 ** -7
    disc = ((math.pi * h / 2) / math.sin(math.pi * h / 2)) ** 2 - 1.0
    out["poisson2d_129_b16"] = dict(ms_per_solve=ms, dof_per_s=127 ** 2 / (ms * 1e-3),
                                    err_vs_fp64=_rel(u[0], ref[0]), plain_fp64_ms_per_solve=pms,
                                    plain_fp64_err_vs_fp64=_rel(up[0], ref[0]), disc_rel_sine_part=disc,
                                    note="errors: relative L2 against a converged float64 solve; disc_rel_sine_part "
                                         "= c_h - 1, the relative discretisation error of the noise-free problem")
    # config 2: 3-D 257^3 sine problem (closed-form discrete solution)
    f = torch.from_numpy(synthetic.sine_rhs(3, 8)).cuda()[None].contiguous()
    for b in (8, 12, 16):
        with Solver(3, 8, smoother="rbgs", bfp_block=64, bits=b) as s:
            ms, u = _time_solves(s, f, 10)
        e, dv = discretisation_check(u[0], 8)
        out[f"poisson3d_257_b{b}"] = dict(ms_per_solve=ms, dof_per_s=255 ** 3 / (ms * 1e-3), err_over_disc=e,
                                          dev_over_disc=dv)
    # config 4: diffusion 129^3, forward + adjoint + gradient
    c4 = W["diffusion3d_129"]
    L = c4["L"]
    kap = torch.from_numpy(synthetic.lognormal_kappa(3, L, c4["kappa_corr"], c4["kappa_seed"])).cuda()
    kobs = torch.from_numpy(synthetic.lognormal_kappa(3, L, c4["kappa_corr"], c4["kappa_obs_seed"])).cuda()
    f = torch.zeros((1,) + ((1 << L) + 1,) * 3, dtype=torch.float64, device="cuda")
    f[:, 1:-1, 1:-1, 1:-1] = 1.0
    uobs = _converged(3, L, f, op="diffusion", kappa=kobs)
    uref = _converged(3, L, f, op="diffusion", kappa=kap)
    with Solver(3, L, op="diffusion", kappa=kap, batch=1, storage="plain", vcycle_prec="fp64",
                final_iters=30) as s:
        lref, gref = s.adjoint(uref, uref - uobs)
    u2h = _converged(3, L - 1, f[:, ::2, ::2, ::2].contiguous(), op="diffusion", kappa=_coarsen_cells(kap))
    with Solver(3, L, op="diffusion", kappa=kap, bits=16, ir_iters=c4["ir_iters"]) as s:
        ms, u = _time_solves(s, f, 5)
        ams, (lam, grad) = _timed(lambda: s.adjoint(u, u - uobs), 3)
    disc4 = _richardson(uref[0], u2h[0])
    out["diffusion3d_129_b16"] = dict(ms_per_solve=ms, dof_per_s=127 ** 3 / (ms * 1e-3), ir_iters=c4["ir_iters"],
                                      ms_adjoint_and_gradient=ams, err_vs_fp64=_rel(u[0], uref[0]),
                                      adjoint_err_vs_fp64=_rel(lam[0], lref[0]), grad_err_vs_fp64=_rel(grad, gref),
                                      disc_rel_richardson=disc4, err_over_disc=_rel(u[0], uref[0]) / disc4,
                                      note="J = 1/2 |u - u_obs|^2; errors relative L2 against converged float64 "
                                           "solves; disc_rel_richardson = |u_h - u_2h| / 3 / |u_h| at coincident "
                                           "nodes (2h: children-mean kappa, same f)")
    del kap, kobs, uobs, uref, lref, gref, u2h, u, lam, grad
    # config 5: diffusion 513^3 x 8, batched forward + adjoint
    c5 = W["diffusion3d_513x8"]
    L, seeds, B = c5["L"], c5["rhs_seeds"], len(c5["rhs_seeds"])
    kap = synthetic.lognormal_kappa_torch(3, L, c5["kappa_corr"], c5["kappa_seed"], device="cuda")
    kobs = synthetic.lognormal_kappa_torch(3, L, c5["kappa_corr"], c5["kappa_obs_seed"], device="cuda")
    f = torch.stack([synthetic.smoothed_noise_rhs_torch(3, L, sd, device="cuda") for sd in seeds])
    log("[bench] diffusion 513^3 x 8: converged float64 references")
    uobs = _converged(3, L, f, op="diffusion", kappa=kobs)
    del kobs
    uref = _converged(3, L, f, op="diffusion", kappa=kap)
    with Solver(3, L, op="diffusion", kappa=kap, batch=B, storage="plain", vcycle_prec="fp64", final_iters=30) as s:
        lref, _ = s.adjoint(uref, uref - uobs, want_grad=False)
    u2h = _converged(3, L - 1, f[:, ::2, ::2, ::2].contiguous(), op="diffusion", kappa=_coarsen_cells(kap))
    disc5 = [_richardson(uref[b], u2h[b]) for b in range(B)]
    del u2h
    with Solver(3, L, op="diffusion", kappa=kap, batch=B, bits=16, ir_iters=c5["ir_iters"]) as s:
        ms, u = _time_solves(s, f, 2)
        dJ = u - uobs
        ams, (lam, _) = _timed(lambda: s.adjoint(u, dJ), 1)
        # one more solve with every kernel timed: the dominant kernel's
        # algorithmic bytes over its launch time, against the HBM peak
        s.timing(True)
        s.solve(f, u)
        torch.cuda.synchronize()
        top = s.timing_report()[0]
        s.timing(False)
    gbs = top["bytes"] / (top["ms"] * 1e-3)
    meas = stored_diffusion_hbm()
    fwd = [_rel(u[b], uref[b]) for b in range(B)]
    adj = [_rel(lam[b], lref[b]) for b in range(B)]
    out["diffusion3d_513x8_b16"] = dict(ms_per_solve=ms, dof_per_s=B * 511 ** 3 / (ms * 1e-3),
                                        ir_iters=c5["ir_iters"], ms_adjoint_and_gradient=ams,
                                        err_vs_fp64_per_rhs=fwd, adjoint_err_vs_fp64_per_rhs=adj,
                                        disc_rel_richardson_per_rhs=disc5,
                                        max_err_over_disc=max(e / d for e, d in zip(fwd, disc5)),
                                        dominant_kernel=dict(kernel=top["kernel"], ms_per_solve=top["ms"],
                                                             launches=top["launches"], gbs=gbs / 1e9,
                                                             hbm_frac=gbs / HBM_PEAK),
                                        measured_hbm=None if meas is None else dict(
                                            gbs=meas, frac=meas * 1e9 / HBM_PEAK,
                                            source="profiles/hbm_traffic_diffusion3d_513x8.md",
                                            note="FETCH_SIZE + WRITE_SIZE (calibrated) over the library's "
                                                 "kernels of one right-hand side's solve, over their summed "
                                                 "duration"),
                                        note="errors relative L2 against converged float64 solves of the same "
                                             "system; the right-hand sides vary on the grid scale, so the "
                                             "Richardson estimate (2h: children-mean kappa, injected f) is a "
                                             "scale, not a converged discretisation error")
    return out


def pmc_pass_diffusion():
    """For counter and trace runs of the compact 513^3 x 8 diffusion workload
    of other_workloads, one right-hand side of it (the batch solves its
    right-hand sides one after another, each with the same kernels): one
    warm-up solve, a calibration copy of CALIB_BYTES, one measured solve;
    no JSON."""
    import torch

    import synthetic
    from paper_2511_19036_amd import Solver
    c5 = synthetic.WORKLOADS["diffusion3d_513x8"]
    L, seed = c5["L"], c5["rhs_seeds"][0]
    kap = synthetic.lognormal_kappa_torch(3, L, c5["kappa_corr"], c5["kappa_seed"], device="cuda")
    f = synthetic.smoothed_noise_rhs_torch(3, L, seed, device="cuda")[None].contiguous()
    with Solver(3, L, op="diffusion", kappa=kap, batch=1, bits=16, ir_iters=c5["ir_iters"]) as s:
        u = torch.empty_like(f)
        s.solve(f, u)
        torch.cuda.synchronize()
        log("[bench] diffusion pmc pass: warm-up solve done")
        a = torch.empty(CALIB_BYTES_DIFF // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # the runtime's copy kernel: CALIB_BYTES_DIFF read and written
        torch.cuda.synchronize()
        del a, b
        s.solve(f, u)
        torch.cuda.synchronize()
    log("[bench] diffusion pmc pass done")


def summarize_diffusion_counters(d):
    """Markdown table of the measured HBM traffic of one right-hand side of
    the compact 513^3 x 8 diffusion workload from directory d: dfetch_ and dwrite_
    counter_collection.csv (FETCH_SIZE, WRITE_SIZE passes of
    --pmc-pass-diffusion) and dkt_kernel_trace.csv (a kernel trace of the
    same command).  Rows after the calibration copy (the measured solve);
    bytes calibrated against the copy as in summarize_counters; per kernel
    (template arguments kept, call arguments dropped) and in total, for the
    library's kernels (the counter passes see only those)."""
    import csv
    import collections

    def load(name):
        return list(csv.DictReader(open(os.path.join(d, name))))

    # the calibration copy: the copy whose WRITE_SIZE is CALIB_BYTES_DIFF;
    # the passes run the same program, so its dispatch id is theirs too
    wrows = load("dwrite_counter_collection.csv")
    calib_row = min((r for r in wrows if "copyBuffer" in r["Kernel_Name"]),
                    key=lambda r: abs(float(r["Counter_Value"]) * 1024.0 - CALIB_BYTES_DIFF))
    cid = int(calib_row["Dispatch_Id"])

    def after_copy(rows):
        copies = [r for r in rows if int(r["Dispatch_Id"]) == cid]
        return copies, [r for r in rows if int(r["Dispatch_Id"]) > cid and "cmg::" in r["Kernel_Name"]]

    def duration(r):
        return int(r["End_Timestamp"]) - int(r["Start_Timestamp"])

    def short(name):
        name = name[5:] if name.startswith("void ") else name
        depth = 0
        for i, ch in enumerate(name):
            depth += ch == "<"
            depth -= ch == ">"
            if ch == "(" and depth == 0:
                return name[:i]
        return name

    scale, calib, acc = {}, {}, collections.defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    for pas, col in (("dfetch", 1), ("dwrite", 2)):
        copies, rows = after_copy(load(f"{pas}_counter_collection.csv"))
        c = float(copies[0]["Counter_Value"])
        calib[pas], scale[pas] = c, CALIB_BYTES_DIFF / (c * 1024.0)
        for r in rows:
            a = acc[short(r["Kernel_Name"])]
            a[col] += float(r["Counter_Value"]) * 1024.0 * scale[pas]
            if col == 1:
                a[0] += 1
    copies, trace = after_copy(load("dkt_kernel_trace.csv"))
    assert copies and "copyBuffer" in copies[0]["Kernel_Name"], "the trace is not a run of the same program"
    for r in trace:
        acc[short(r["Kernel_Name"])][3] += duration(r) * 1e-9
    tb = sum(a[1] + a[2] for a in acc.values())
    tt = sum(a[3] for a in acc.values())
    out = [f"measured_gbs: {tb / tt / 1e9:.1f}",
           f"source_sha256_all: {kernel_source_digest(ALL_SOURCES)}",
           "",
           f"Calibration: the runtime's copy of {CALIB_BYTES_DIFF} bytes reads FETCH_SIZE = {calib['dfetch']:.1f} KiB "
           f"and WRITE_SIZE = {calib['dwrite']:.1f} KiB (scales {scale['dfetch']:.4f}, {scale['dwrite']:.4f}).",
           "",
           f"Measured solve (one right-hand side): {tb / 1e9:.2f} GB of HBM traffic in {tt * 1e3:.1f} ms of "
           f"kernel time: "
           f"{tb / tt / 1e9:.0f} GB/s, {tb / tt / HBM_PEAK:.1%} of {HBM_PEAK / 1e12:.0f} TB/s.",
           "",
           "| kernel | launches | HBM GB (calibrated) | kernel ms | GB/s | of peak |",
           "|---|---:|---:|---:|---:|---:|"]
    for k, a in sorted(acc.items(), key=lambda kv: -kv[1][3]):
        if a[3] <= 0 or a[3] < 0.005 * tt:
            continue
        gb = (a[1] + a[2]) / 1e9
        out.append(f"| `{k}` | {a[0]} | {gb:.2f} | {a[3] * 1e3:.1f} | {gb / a[3]:.0f} | "
                   f"{gb * 1e9 / a[3] / HBM_PEAK:.1%} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=10)
    ap.add_argument("--bits", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 FMG comparison")
    ap.add_argument("--cpu-L", type=int, default=8)
    ap.add_argument("--cpu-procs", type=int, default=16, help="oracle processes for the all-core CPU rate")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 8/12-bit and tuned-width runs")
    ap.add_argument("--no-workloads", action="store_true", help="skip the timings of the other workloads")
    ap.add_argument("--no-codec", action="store_true", help="skip the adaptive-exponent codec timing")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for counter runs: one warm-up solve, a calibration copy of 1 GiB, one solve; no JSON")
    ap.add_argument("--only-workloads", action="store_true",
                    help="for kernel traces: time only the other workloads and print their figures as JSON")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="print the markdown tables of the --pmc-pass counter csv files in DIR (no GPU)")
    ap.add_argument("--summarize-stalls", metavar="DIR",
                    help="print the markdown table of the SQ stall counter csv files (passes sa_, sb_) in DIR "
                         "(no GPU)")
    ap.add_argument("--pmc-pass-diffusion", action="store_true",
                    help="for counter and trace runs: one right-hand side of the 513^3 x 8 diffusion workload, "
                         "warm-up, copy, one solve")
    ap.add_argument("--summarize-diffusion", metavar="DIR",
                    help="print the measured HBM table of the --pmc-pass-diffusion csv files in DIR (no GPU)")
    args = ap.parse_args()
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.L, args.bits))
        return
    if args.summarize_stalls:
        print(summarize_stalls(args.summarize_stalls, args.L, args.bits))
        return
    if args.summarize_diffusion:
        print(summarize_diffusion_counters(args.summarize_diffusion))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the solver is a single-GPU level sweep); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.only_workloads:
        print(json.dumps(other_workloads()), flush=True)
        return
    if args.pmc_pass_diffusion:
        pmc_pass_diffusion()
        return

    import torch

    import synthetic
    from paper_2511_19036_amd import Solver

    L, dim = args.L, 3
    N = (1 << L) + 1
    dofs = ((1 << L) - 1) ** 3
    log(f"[bench] building f on the GPU: {N}^3 nodes")
    f = synthetic.hash_noise_rhs_torch(dim, L, amp=1e-4, seed=3, device="cuda")[None].contiguous()
    torch.cuda.synchronize()

    log(f"[bench] setup compact solver (b={args.bits}, B=64)")
    t0 = time.perf_counter()
    s = Solver(dim, L, smoother="rbgs", bfp_block=64, bits=args.bits, ir_iters=2, vcycle_prec="fp32")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    u = torch.empty_like(f)
    if args.pmc_pass:
        s.solve(f, u)
        a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # device-to-device copy: the runtime's copy kernel, CALIB_BYTES read and written
        torch.cuda.synchronize()
        s.solve(f, u)
        torch.cuda.synchronize()
        log("[bench] pmc pass done")
        return
    for w in range(args.warmup):
        s.solve(f, u)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")

    # one untimed solve with every kernel timed per level: the dominant kernel
    s.timing(True, "@")
    s.solve(f, u)
    torch.cuda.synchronize()
    per_level = s.timing_report()
    s.timing(False)
    per_kernel = _by_kernel(per_level)
    dom = per_kernel[0]["kernel"]
    log(f"[bench] dominant kernel: {dom} ({per_kernel[0]['ms']:.2f} ms of "
        f"{sum(r['ms'] for r in per_kernel):.2f} ms per solve)")

    # timed region: K solves; HIP events bracket the dominant kernel's
    # launches on the finest level
    s.timing(True, f"{dom}@{L}")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        s.solve(f, u)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    rep = [r for r in s.timing_report() if r["kernel"] == dom][0]
    s.timing(False)
    log(f"[bench] compact FMG: {ms:.2f} ms per solve")

    err_disc, dev_disc = discretisation_check(u[0], L)
    mem = s.memory_stats()
    s.close()
    del s

    codec = None if args.no_codec else codec_rates(u.view(-1), args.bits)

    # Roofline of the dominant kernel on the finest level: its algorithmic
    # bytes per interior DoF at the finest widths (the survey's per-DoF
    # model, logical widths), times the DoF of one launch, over the average
    # launch time measured with HIP events inside the timed solves.
    bpd = model_bytes_per_dof(dom, args.bits, 64)
    avg_s = 1e-3 * rep["ms"] / rep["launches"]
    achieved = bpd * dofs / avg_s
    traffic = stored_traffic(f"{dom}@{L}")
    levels = []
    for r in per_level:
        name, _, lv = r["kernel"].partition("@")
        if name == dom and lv:
            lvl = int(lv)
            levels.append(dict(level=lvl, launches=r["launches"], avg_launch_us=1e3 * r["ms"] / r["launches"],
                               library_bytes_per_launch=r["bytes"] / r["launches"],
                               library_gbs=r["bytes"] / (r["ms"] * 1e-3) / 1e9,
                               library_frac=r["bytes"] / (r["ms"] * 1e-3) / HBM_PEAK))
    levels.sort(key=lambda d: -d["level"])
    dom_all = [r for r in per_kernel if r["kernel"] == dom][0]
    roofline = dict(bound="hbm", kernel=dom, level=L, achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / HBM_PEAK, traffic=traffic, bytes_per_dof=bpd, dofs_per_launch=dofs,
                    bytes_per_launch=bpd * dofs, avg_launch_us=1e6 * avg_s, launches=rep["launches"],
                    per_level=levels,
                    all_levels_library_count=dict(
                        note="every level's launches together, bytes as the library counts them (section "
                             "containers, e.g. 17-24-bit codes in 32-bit words)",
                        gbs=dom_all["bytes"] / (dom_all["ms"] * 1e-3) / 1e9,
                        frac=dom_all["bytes"] / (dom_all["ms"] * 1e-3) / HBM_PEAK))
    # All fused level kernels of one solve together (from the per-kernel
    # timing pass): algorithmic bytes and, from the stored counter readings,
    # measured HBM bytes over their summed launch time.
    fams = ("k_up_smooth<4>", "k_down_smooth<4>", "k_ir_residual", "k_resid_restrict", "k_decode_full",
            "k_decode_level")
    sweep_rows = [r for r in per_kernel if r["kernel"] in fams]
    sweep_s = sum(r["ms"] for r in sweep_rows) * 1e-3
    sweep_alg = sum(r["bytes"] for r in sweep_rows)
    hbm = [stored_traffic(r["kernel"]) for r in sweep_rows]
    sweep_hbm = sum(h * r["launches"] for h, r in zip(hbm, sweep_rows)) if all(h is not None for h in hbm) else None
    level_sweep = dict(kernels=[r["kernel"] for r in sweep_rows], ms_per_solve=sweep_s * 1e3,
                       algorithmic_gbs=sweep_alg / sweep_s / 1e9, algorithmic_frac=sweep_alg / sweep_s / HBM_PEAK,
                       measured_gbs=None if sweep_hbm is None else sweep_hbm / sweep_s / 1e9,
                       measured_frac=None if sweep_hbm is None else sweep_hbm / sweep_s / HBM_PEAK)
    # the same kernel against its instruction-issue ceiling: counted VALU
    # instructions per finest-level launch over the live average launch time
    valu = stored_valu(f"{dom}@{L}")
    issue = None
    if valu is not None:
        issue = dict(kernel=dom, level=L, valu_insts_per_launch=valu, peak_insts_per_s=VALU_PEAK,
                     frac=valu / VALU_PEAK / avg_s)

    plain = None
    if not args.no_plain:
        log("[bench] plain FP64 FMG comparison")
        p = Solver(dim, L, smoother="rbgs", storage="plain", vcycle_prec="fp64", ir_iters=2)
        p.solve(f, u)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps_p = max(1, min(args.steps, 3))
        e0.record()
        for _ in range(steps_p):
            p.solve(f, u)
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / steps_p
        perr, pdev = discretisation_check(u[0], L)
        pmem = p.memory_stats()
        p.close()
        plain = dict(dof_per_s=dofs / (pms * 1e-3), ms_per_solve=pms, err_over_disc=perr, dev_over_disc=pdev,
                     bytes_per_dof=pmem["total"] / dofs)

    def solve_rate(opts, steps):
        """DoF/s, accuracy and bytes/DoF of the same problem with other widths."""
        q = Solver(dim, L, smoother="rbgs", bfp_block=64, vcycle_prec="fp32", **opts)
        q.solve(f, u)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            q.solve(f, u)
        e1.record()
        torch.cuda.synchronize()
        qms = e0.elapsed_time(e1) / steps
        qerr, qdev = discretisation_check(u[0], L)
        qmem = q.memory_stats()
        q.close()
        return dict(opts=opts, dof_per_s=dofs / (qms * 1e-3), ms_per_solve=qms, err_over_disc=qerr,
                    dev_over_disc=qdev, accuracy_pass=bool(qerr <= 2.0 and qdev <= 0.5),
                    bytes_per_dof=qmem["total"] / dofs, logical_bits_per_dof=qmem["logical_bits_per_dof"])

    sweep = None
    if not args.no_sweep:
        sweep = {}
        for b in (8, 12):
            log(f"[bench] compact FMG with {b}-bit tails")
            sweep[str(b)] = solve_rate(dict(bits=b, ir_iters=2), min(args.steps, 3))
        from paper_2511_19036_amd.tune import tune_widths
        log("[bench] tuning widths and N on the 33^3 .. 65^3 sine problems (Sec. 7.1 procedure)")
        t0 = time.perf_counter()
        tuned = tune_widths(3, 6, smoother="rbgs", omega=1.0, bfp_block=64)
        tune_s = time.perf_counter() - t0
        log(f"[bench] tuned: {tuned} ({tune_s:.1f} s); timing it at {N}^3")
        sweep["tuned"] = solve_rate(tuned, min(args.steps, 3))
        sweep["tuned"]["tuning_s"] = tune_s

    others = None
    if not args.no_workloads:
        others = other_workloads()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU baseline: oracle at {(1 << args.cpu_L) + 1}^3")
        cpu = cpu_baseline(args.cpu_L, args.bits, max(1, min(args.cpu_procs, os.cpu_count() or 1)))

    out = {
        "metric": "DoF/s solved to discretization error; bytes/DoF; HBM GB/s vs peak",
        "value": dofs / (ms * 1e-3),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"3-D Poisson 7-point FD, {N}^3 nodes, f = 3 pi^2 sin sin sin + 1e-4 U[-1,1) "
                        f"(hashed, seed 3); compact FMG N=2, V(2,2) RB-GS FP32, FP64 IR residual",
            "dofs": dofs, "bits": args.bits, "bfp_block": 64, "storage": "compact",
            "parallelism": "single GPU",
        },
        "accuracy": {"err_over_disc": err_disc, "dev_over_disc": dev_disc,
                     "pass": bool(err_disc <= 2.0 and dev_disc <= 0.5)},
        "bytes_per_dof": mem["total"] / dofs,
        "logical_bits_per_dof": mem["logical_bits_per_dof"],
        "setup_s": setup_s,
        "roofline": roofline,
        "issue": issue,
        "level_sweep": level_sweep,
        "kernels": [dict(kernel=r["kernel"], ms=r["ms"], launches=r["launches"],
                         gbs=(r["bytes"] / (r["ms"] * 1e-3) / 1e9) if r["ms"] > 0 else None)
                    for r in per_kernel[:12]],
        "plain_fp64": plain,
        "width_sweep": sweep,
        "other_workloads": others,
        "cpu_baseline": cpu,
        "adaptive_bfp": codec,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
