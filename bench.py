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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest():
    """SHA-256 of the fused-kernel sources (fused.hip and the device headers
    it includes) with comments and blank lines removed, to tell whether
    stored counter readings still describe the kernels being run."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("fused.hip", "plane.h", "device.h"):
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


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    against a copy of known size) from the committed counter summary."""
    return _stored_column("hbm_traffic_fused_kernels_poisson3d_1025.md", kernel, 5)


def stored_valu(kernel):
    """VALU wave instructions per launch of `kernel` (SQ_INSTS_VALU) from the
    committed counter summary."""
    return _stored_column("valu_issue_fused_kernels_poisson3d_1025.md", kernel, 2)


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


def cpu_baseline(L_sample: int, bits: int):
    """The oracle (numpy, as it stands) on the same problem at a smaller grid."""
    import numpy as np  # noqa: F401

    import synthetic
    from oracle import compact as oc
    f = synthetic.hash_noise_rhs(3, L_sample, amp=1e-4, seed=3)
    cfg = oc.Config(dim=3, L=L_sample, smoother="rbgs", omega=1.0, block=64,
                    bits_u=bits, bits_r=bits, bits_y=bits)
    t = time.perf_counter()
    oc.fmg_solve(f, cfg)
    t = time.perf_counter() - t
    dofs = ((1 << L_sample) - 1) ** 3
    return dict(value=dofs / t, unit="DoF/s", cores=1, kind="oracle",
                sample=f"the same problem and solver settings at {(1 << L_sample) + 1}^3 "
                       f"({dofs} DoF), one FMG solve, {t:.1f} s on one host thread")


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


def other_workloads():
    """Solve times of the other workloads (same library, same GPU)."""
    import torch

    import synthetic
    from paper_2511_19036_amd import Solver
    out = {}
    log("[bench] other workloads: 2-D 129^2, 3-D 257^3, diffusion 129^3 and 513^3 x 8")
    f = torch.from_numpy(synthetic.gaussian_noise_rhs(2, 7, 1e-3, 0)).cuda()[None].contiguous()
    with Solver(2, 7, smoother="wjacobi", omega=0.8, bfp_block=32, bits=16) as s:
        ms, _ = _time_solves(s, f, 20)
    out["poisson2d_129_b16"] = dict(ms_per_solve=ms, dof_per_s=127 ** 2 / (ms * 1e-3))
    f = torch.from_numpy(synthetic.sine_rhs(3, 8)).cuda()[None].contiguous()
    for b in (8, 12, 16):
        with Solver(3, 8, smoother="rbgs", bfp_block=64, bits=b) as s:
            ms, u = _time_solves(s, f, 10)
        e, dv = discretisation_check(u[0], 8)
        out[f"poisson3d_257_b{b}"] = dict(ms_per_solve=ms, dof_per_s=255 ** 3 / (ms * 1e-3), err_over_disc=e,
                                          dev_over_disc=dv)
    kap = torch.from_numpy(synthetic.lognormal_kappa(3, 7, 0.1, 1)).cuda()
    f = torch.zeros((1, 129, 129, 129), dtype=torch.float64, device="cuda")
    f[:, 1:-1, 1:-1, 1:-1] = 1.0
    with Solver(3, 7, op="diffusion", kappa=kap, bits=16) as s:
        ms, u = _time_solves(s, f, 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.adjoint(u, u)
        e1.record()
        torch.cuda.synchronize()
    out["diffusion3d_129_b16"] = dict(ms_per_solve=ms, dof_per_s=127 ** 3 / (ms * 1e-3),
                                      ms_adjoint_and_gradient=e0.elapsed_time(e1))
    kap = synthetic.lognormal_kappa_torch(3, 9, 0.05, 4, device="cuda")
    f = torch.stack([synthetic.smoothed_noise_rhs_torch(3, 9, sd, device="cuda") for sd in range(100, 108)])
    with Solver(3, 9, op="diffusion", kappa=kap, batch=8, bits=16) as s:
        ms, u = _time_solves(s, f, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.adjoint(u, u)
        e1.record()
        torch.cuda.synchronize()
        # one more solve with every kernel timed: the dominant kernel's
        # algorithmic bytes over its launch time, against the HBM peak
        s.timing(True)
        s.solve(f, u)
        torch.cuda.synchronize()
        top = s.timing_report()[0]
        s.timing(False)
    gbs = top["bytes"] / (top["ms"] * 1e-3)
    out["diffusion3d_513x8_b16"] = dict(ms_per_solve=ms, dof_per_s=8 * 511 ** 3 / (ms * 1e-3),
                                        ms_adjoint_and_gradient=e0.elapsed_time(e1),
                                        dominant_kernel=dict(kernel=top["kernel"], ms_per_solve=top["ms"],
                                                             launches=top["launches"], gbs=gbs / 1e9,
                                                             hbm_frac=gbs / HBM_PEAK),
                                        note="diffusion runs the per-operation kernels (one launch per red-black "
                                             "sweep; the fused level kernels are Poisson-only)")
    return out


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
    ap.add_argument("--no-sweep", action="store_true", help="skip the 8/12-bit and tuned-width runs")
    ap.add_argument("--no-workloads", action="store_true", help="skip the timings of the other workloads")
    ap.add_argument("--no-codec", action="store_true", help="skip the adaptive-exponent codec timing")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for counter runs: one warm-up solve, a calibration copy of 1 GiB, one solve; no JSON")
    ap.add_argument("--only-workloads", action="store_true",
                    help="for kernel traces: time only the other workloads and print their figures as JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the solver is a single-GPU level sweep); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.only_workloads:
        print(json.dumps(other_workloads()), flush=True)
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

    # one untimed solve with every kernel timed: find the dominant kernel
    s.timing(True)
    s.solve(f, u)
    torch.cuda.synchronize()
    per_kernel = s.timing_report()
    dom = per_kernel[0]["kernel"]
    log(f"[bench] dominant kernel: {dom} ({per_kernel[0]['ms']:.2f} ms of "
        f"{sum(r['ms'] for r in per_kernel):.2f} ms per solve)")

    # timed region: K solves; HIP events bracket the dominant kernel's launches
    s.timing(True, dom)
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

    achieved = rep["bytes"] / (rep["ms"] * 1e-3)
    traffic = stored_traffic(dom)
    roofline = dict(bound="hbm", kernel=dom, achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / HBM_PEAK, traffic=traffic,
                    bytes_per_launch=rep["bytes"] / rep["launches"],
                    avg_launch_us=1e3 * rep["ms"] / rep["launches"], launches=rep["launches"])
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
    # instructions per launch over the live average launch time
    valu = stored_valu(dom)
    issue = None
    if valu is not None:
        avg_s = 1e-3 * rep["ms"] / rep["launches"]
        issue = dict(kernel=dom, valu_insts_per_launch=valu, peak_insts_per_s=VALU_PEAK,
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
        cpu = cpu_baseline(args.cpu_L, args.bits)

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
