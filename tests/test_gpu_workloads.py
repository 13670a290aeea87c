"""The benchmark workloads at their own sizes (beyond what the oracle can run).

* 3-D Poisson, 257^3 nodes, u* = prod sin(pi x_i), red-black Gauss-Seidel
  V(2,2), BFP block 64, 8/12/16-bit tails: the compact FMG meets the
  paper's acceptance test (error at most twice the discretisation error)
  and converges at order >= 1.95 over 33^3 .. 257^3.
* 3-D variable-coefficient diffusion, 513^3 nodes, log-normal kappa
  (correlation length 0.05, unit variance), 8 seeded smoothed-noise
  right-hand sides (drawn on the device at this size): the batched solve
  equals the per-item solves exactly, and against a converged float64
  solve of the same system (plain storage, float64 V-cycles, 12 extra
  iterations) the compact FMG's error per right-hand side is at most 1.05
  times that of the plain float64 FMG with the same iteration counts, i.e.
  storing the tails in BFP costs no accuracy the float64 multigrid has;
  the small-grid version of the same batch matches the oracle bit for bit.
"""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import compact as oc
from oracle import grid as og

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cmg(gpu_lib):
    import paper_2511_19036_amd
    return paper_2511_19036_amd


def _sine_errors(cmg, L, bits):
    h = 2.0 ** -L
    us = S.sine_solution(3, L)
    uh = ((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2 * us  # exact discrete solution
    with cmg.Solver(3, L, smoother="rbgs", bits=bits, bfp_block=64) as s:
        u = s.solve(torch.from_numpy(S.sine_rhs(3, L)).cuda()[None])[0].cpu().numpy()
    return og.norm_h(u - us, h), og.norm_h(uh - us, h)


@pytest.mark.parametrize("bits", [8, 12, 16])
def test_poisson3d_257_accuracy_and_order(cmg, bits):
    errs = {}
    for L in (5, 6, 7, 8):
        e, disc = _sine_errors(cmg, L, bits)
        assert e <= 2.0 * disc, (L, e, disc)
        errs[L] = e
    for L in (6, 7, 8):
        assert np.log2(errs[L - 1] / errs[L]) >= 1.95, (L, errs)


def _diffusion_batch(L, corr, kseed, seeds):
    kappa = torch.from_numpy(S.lognormal_kappa(3, L, corr, kseed)).cuda()
    f = torch.stack([torch.from_numpy(S.smoothed_noise_rhs(3, L, sd)) for sd in seeds]).cuda()
    return kappa, f


def test_diffusion_batch_matches_oracle_small(cmg):
    L, seeds = 5, (100, 101, 102)
    kappa, f = _diffusion_batch(L, 0.05, 4, seeds)
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), bits=16) as s:
        u = s.solve(f).cpu().numpy()
    cfg = oc.Config(dim=3, L=L, op="diffusion", smoother="rbgs", block=64, bits_u=16, bits_r=16, bits_y=16)
    for b in range(len(seeds)):
        ref, _ = oc.fmg_solve(f[b].cpu().numpy(), cfg, kappa.cpu().numpy())
        assert np.array_equal(u[b], ref), b


@pytest.mark.slow
def test_diffusion3d_513x8_batch(cmg):
    L, seeds = 9, tuple(range(100, 108))
    kappa = S.lognormal_kappa_torch(3, L, 0.05, 4, device="cuda")
    f = torch.stack([S.smoothed_noise_rhs_torch(3, L, sd, device="cuda") for sd in seeds])
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), bits=16) as s:
        u = s.solve(f)
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=1, bits=16) as s:
        for b in (0, len(seeds) - 1):
            assert torch.equal(s.solve(f[b:b + 1].contiguous())[0], u[b]), b
    plain = dict(storage="plain", vcycle_prec="fp64")
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), final_iters=12, **plain) as s:
        ref = s.solve(f)
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), **plain) as s:
        up = s.solve(f)
    for b in range(len(seeds)):
        nr = torch.linalg.vector_norm(ref[b])
        ec = float(torch.linalg.vector_norm(u[b] - ref[b]) / nr)
        ep = float(torch.linalg.vector_norm(up[b] - ref[b]) / nr)
        print(f"rhs {b}: relative L2 error vs converged: compact {ec:.3e}, plain float64 FMG {ep:.3e}", flush=True)
        assert ec <= 1.05 * ep, (b, ec, ep)


@pytest.mark.slow
def test_poisson3d_1025_headline_configuration(cmg):
    """The benchmark's own configuration (1025^3, hashed 1e-4 noise, b = 16,
    B = 64, N = 2, FP32 V-cycle): the solution meets the acceptance test
    against the closed-form discrete solution of the sine part (the noise
    moves it by ~1e-10 relative) and the solver state stays below 13 bytes
    per DoF, a quarter of what plain FP64 multigrid allocates."""
    import math
    L = 10
    f = S.hash_noise_rhs_torch(3, L, amp=1e-4, seed=3, device="cuda")[None].contiguous()
    with cmg.Solver(3, L, smoother="rbgs", bfp_block=64, bits=16, ir_iters=2, vcycle_prec="fp32") as s:
        u = s.solve(f)
        mem = s.memory_stats()
    h = 2.0 ** -L
    N = (1 << L) + 1
    x = torch.arange(N, dtype=torch.float64, device="cuda") * h
    sn = torch.sin(math.pi * x)
    sn[0] = 0.0
    sn[-1] = 0.0
    ch = ((math.pi * h / 2) / math.sin(math.pi * h / 2)) ** 2
    err2 = dev2 = disc2 = 0.0
    for k in range(N):
        us = sn[k] * (sn[:, None] * sn[None, :])
        err2 += float(((u[0, k] - us) ** 2).sum())
        dev2 += float(((u[0, k] - ch * us) ** 2).sum())
        disc2 += float((((ch - 1.0) * us) ** 2).sum())
    assert math.sqrt(err2 / disc2) <= 2.0
    assert math.sqrt(dev2 / disc2) <= 0.5
    assert mem["total"] / 1023 ** 3 < 13.0
