"""The benchmark workloads at their own sizes (beyond what the oracle can run).

* 3-D Poisson, 257^3 nodes, u* = prod sin(pi x_i), red-black Gauss-Seidel
  V(2,2), BFP block 64, 8/12/16-bit tails: the compact FMG meets the
  paper's acceptance test (error at most twice the discretisation error)
  and converges at order >= 1.95 over 33^3 .. 257^3.
* 3-D variable-coefficient diffusion, 513^3 nodes, log-normal kappa
  (correlation length 0.05, unit variance), 8 seeded smoothed-noise
  right-hand sides (drawn on the device at this size), N = 3: the batched
  solve equals the per-item solves exactly; against a converged float64
  solve of the same system (plain storage, float64 V-cycles, 30 extra
  iterations) the compact FMG's error per right-hand side is at most half
  the Richardson estimate of the discretisation error and below 1e-3, and
  at most 1.05 times that of the plain float64 FMG with the same iteration
  counts; the small-grid version of the same batch matches the oracle bit
  for bit.
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


def _coarsen_cells(k):
    n = k.shape[0] // 2
    return k.reshape(n, 2, n, 2, n, 2).mean(dim=(1, 3, 5)).contiguous()


@pytest.mark.slow
def test_diffusion3d_513x8_batch(cmg):
    L, seeds = 9, tuple(range(100, 108))
    N = S.WORKLOADS["diffusion3d_513x8"]["ir_iters"]
    kappa = S.lognormal_kappa_torch(3, L, 0.05, 4, device="cuda")
    f = torch.stack([S.smoothed_noise_rhs_torch(3, L, sd, device="cuda") for sd in seeds])
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), bits=16, ir_iters=N) as s:
        u = s.solve(f)
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=1, bits=16, ir_iters=N) as s:
        for b in (0, len(seeds) - 1):
            assert torch.equal(s.solve(f[b:b + 1].contiguous())[0], u[b]), b
    plain = dict(storage="plain", vcycle_prec="fp64")
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), final_iters=30, **plain) as s:
        ref = s.solve(f)
    with cmg.Solver(3, L, op="diffusion", kappa=kappa, batch=len(seeds), ir_iters=N, **plain) as s:
        up = s.solve(f)
    # discretisation-error scale: Richardson from the same system on 2h
    # (children-mean kappa, injected right-hand side), at coincident nodes
    with cmg.Solver(3, L - 1, op="diffusion", kappa=_coarsen_cells(kappa), batch=len(seeds), final_iters=30,
                    **plain) as s:
        ref2 = s.solve(f[:, ::2, ::2, ::2].contiguous())
    for b in range(len(seeds)):
        nr = torch.linalg.vector_norm(ref[b])
        ec = float(torch.linalg.vector_norm(u[b] - ref[b]) / nr)
        ep = float(torch.linalg.vector_norm(up[b] - ref[b]) / nr)
        c = ref[b][::2, ::2, ::2]
        disc = float(torch.linalg.vector_norm(c - ref2[b]) / 3.0 / torch.linalg.vector_norm(c))
        print(f"rhs {b}: relative L2 error vs converged: compact {ec:.3e}, plain float64 FMG {ep:.3e}; "
              f"Richardson discretisation estimate {disc:.3e}", flush=True)
        # the paper's acceptance reading: the solver error is at most half
        # the discretisation error (measured 0.05x at N = 3), and absolutely
        # below 1e-3 (measured 1.7e-4 .. 3.0e-4)
        assert ec <= 0.5 * disc and ec <= 1e-3, (b, ec, disc)
        assert ec <= 1.05 * ep + 1e-6, (b, ec, ep)


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


@pytest.mark.slow
def test_poisson3d_1025_ir_residual_sampled_blocks(cmg):
    """Alg. 2 at full size, in the configuration bench.py times (1025^3,
    b = 16, B = 64, the fused float64 residual kernel): random compact
    sections are imported on every level, one IR residual runs on the GPU,
    and sampled residual blocks (boundary rows included) equal the
    node-by-node oracle bit for bit; so do 109 sampled nodes of the final
    decode (eq. compact-to-standard) of the same sections."""
    from oracle import bfp as ob
    from oracle import pointwise as pw
    L, B = 10, 64
    n = 1 << L
    f = S.hash_noise_rhs_torch(3, L, amp=1e-4, seed=3, device="cuda")[None].contiguous()
    rng = np.random.default_rng(21)
    Uc = {}
    dtypes = {8: np.int8, 16: np.int16, 32: np.int32, 64: np.int64}
    with cmg.Solver(3, L, smoother="rbgs", bfp_block=B, bits=16, ir_iters=2, vcycle_prec="fp32") as s:
        for level in range(1, L + 1):
            s.enter_level(level, f)
        for level in range(1, L + 1):
            w = s.section_info("u", level)["bits"]
            m = 1 << level
            lim = (1 << (w - 1)) - 1
            nblk = (m ** 3 + B - 1) // B                     # sections hold whole blocks
            codes = np.zeros(nblk * B, dtype=dtypes[ob.container_bits(w)])
            codes[: m ** 3] = rng.integers(-lim, lim + 1, size=m ** 3, dtype=codes.dtype)
            c3 = codes[: m ** 3].reshape(m, m, m)
            c3[0], c3[:, 0], c3[:, :, 0] = 0, 0, 0          # Dirichlet nodes hold 0
            exps = rng.integers(-2 * level - 6, -2 * level + 3, size=nblk, dtype=np.int16)
            s.import_section("u", level, w, codes.view(np.uint8), exps)
            Uc[level] = pw.Codes(codes, exps, B, w)
        s.ir_residual(f)
        gcodes, gexps, gw = s.export_section("r", L)
        # the final decode (k_decode_full) of the same sections: sampled
        # nodes of the full node grid, far faces and edges included
        u = s.decode_solution(L)
        pts = [(0, 0, 0), (n, n, n), (n, 5, 7), (3, n, 9), (11, 13, n), (1, 1, 1), (n - 1, n - 1, n - 1),
               (n - 1, 1, n), (2, n - 1, 1)]
        pts += [tuple(int(v) for v in r) for r in rng.integers(0, n + 1, (100, 3))]
        idx = np.array(pts, dtype=np.int64)
        got = u[tuple(torch.from_numpy(idx[:, a]).cuda() for a in range(3))].cpu().numpy()
        del u
    want = pw.decode_chain_at(Uc, 1, L, idx)
    assert np.array_equal(got, want)
    assert ob.container_bits(gw) == 16
    gm = gcodes.view(np.int16).reshape(n, n, n // B, B)
    ge = gexps.reshape(n, n, n // B)
    rows = [(0, 3, 0), (5, 0, 2), (1, 1, 0), (n - 1, n - 1, n // B - 1), (n - 1, 1, 0)]
    rows += [tuple(int(v) for v in r) for r in np.stack([rng.integers(0, n, 150), rng.integers(0, n, 150),
                                                         rng.integers(0, n // B, 150)], axis=1)]
    for z, y, bx in rows:
        fb = f[0, z, y, bx * B:(bx + 1) * B].cpu().numpy()
        mo, eo = pw.ir_residual_block(Uc, 1, L, fb, z, y, bx, B, gw)
        assert int(ge[z, y, bx]) == eo, (z, y, bx)
        assert np.array_equal(gm[z, y, bx].astype(np.int64), mo), (z, y, bx)


@pytest.mark.slow
def test_poisson3d_1025_down_sweep_sampled_blocks(cmg):
    """The fused down sweep and residual restriction at full size (1025^3,
    b = 16, B = 64, V(2,2)): a random residual section is imported on the
    finest level, one V-cycle runs on the GPU, and sampled blocks of the
    pre-smoothed correction y'_L and of the restricted g_{L-1} (boundary rows
    included) equal the node-local oracle bit for bit."""
    from oracle import bfp as ob
    from oracle import pointwise as pw
    L, B, nu = 10, 64, 2
    n, m = 1 << L, 1 << (L - 1)
    f = torch.zeros((1,) + ((n + 1),) * 3, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(31)
    with cmg.Solver(3, L, smoother="rbgs", bfp_block=B, bits=16, ir_iters=2, vcycle_prec="fp32",
                    keep_correction=True) as s:
        for level in range(1, L + 1):
            s.enter_level(level, f)
        w = s.section_info("r", L)["bits"]
        assert ob.container_bits(w) == 16
        lim = (1 << (w - 1)) - 1
        codes = rng.integers(-lim, lim + 1, size=n ** 3, dtype=np.int16)
        c3 = codes.reshape(n, n, n)
        c3[0], c3[:, 0], c3[:, :, 0] = 0, 0, 0              # Dirichlet nodes hold 0
        exps = rng.integers(-3, 4, size=n ** 3 // B, dtype=np.int16)
        s.import_section("r", L, w, codes.view(np.uint8), exps)
        s.vcycle_correct()
        ym, ye, yw = s.export_section("ypre", L)
        gm, ge, gw = s.export_section("r", L - 1)
    del f
    G = pw.Codes(codes, exps, B, w)
    ym = ym.view(np.int16).reshape(n, n, n // B, B)
    ye = ye.reshape(n, n, n // B)
    rows = [(0, 3, 0), (1, 1, 0), (n - 1, n - 1, n // B - 1), (2, n - 1, 3), (n - 1, 1, 5)]
    rows += [tuple(int(v) for v in r) for r in np.stack([rng.integers(0, n, 40), rng.integers(0, n, 40),
                                                         rng.integers(0, n // B, 40)], axis=1)]
    for z, y, bx in rows:
        mo, eo = pw.down_sweep_block(G, L, nu, z, y, bx, B, yw)
        assert int(ye[z, y, bx]) == eo, (z, y, bx)
        assert np.array_equal(ym[z, y, bx].astype(np.int64), mo), (z, y, bx)
    dt = {8: np.int8, 16: np.int16, 32: np.int32, 64: np.int64}[ob.container_bits(gw)]
    gm = gm.view(dt).reshape(m, m, m // B, B)
    ge = ge.reshape(m, m, m // B)
    crow = [(0, 2, 0), (1, 1, 0), (m - 1, m - 1, m // B - 1), (3, m - 1, 2)]
    crow += [tuple(int(v) for v in r) for r in np.stack([rng.integers(0, m, 25), rng.integers(0, m, 25),
                                                         rng.integers(0, m // B, 25)], axis=1)]
    for K, J, bxc in crow:
        mo, eo = pw.restrict_block(G, L, nu, K, J, bxc, B, yw, gw)
        assert int(ge[K, J, bxc]) == eo, (K, J, bxc)
        assert np.array_equal(gm[K, J, bxc].astype(np.int64), mo), (K, J, bxc)


@pytest.mark.slow
def test_poisson3d_1025_up_sweep_sampled_blocks(cmg):
    """The fused up sweep and correction, the dominant kernel, at full size
    (1025^3, b = 16, B = 64, V(2,2)) in the configuration bench.py times:
    random residual, pre-smoothed correction and solution sections are
    imported on the finest level and a random float32 coarse correction
    e_{L-1} is given; the up sweep of that level runs alone, and sampled
    blocks of the post-smoothed correction y'_L and of the corrected u'_L
    (boundary rows included) equal the node-local oracle bit for bit."""
    from oracle import bfp as ob
    from oracle import pointwise as pw
    L, B, nu = 10, 64, 2
    n, m = 1 << L, 1 << (L - 1)
    f = torch.zeros((1,) + ((n + 1),) * 3, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(41)

    def random_section(w, elo, ehi):
        lim = (1 << (w - 1)) - 1
        codes = rng.integers(-lim, lim + 1, size=n ** 3, dtype=np.int16)
        c3 = codes.reshape(n, n, n)
        c3[0], c3[:, 0], c3[:, :, 0] = 0, 0, 0              # Dirichlet nodes hold 0
        exps = rng.integers(elo, ehi, size=n ** 3 // B, dtype=np.int16)
        return codes, exps

    e_np = np.zeros((m, m, m), dtype=np.float32)
    e_np[1:, 1:, 1:] = rng.uniform(-1e-6, 1e-6, size=(m - 1,) * 3).astype(np.float32)
    with cmg.Solver(3, L, smoother="rbgs", bfp_block=B, bits=16, ir_iters=2, vcycle_prec="fp32",
                    keep_correction=True) as s:
        for level in range(1, L + 1):
            s.enter_level(level, f)
        secs = {}
        for which, (elo, ehi) in (("r", (-3, 4)), ("ypre", (-24, -19)), ("u", (-10, -4))):
            w = s.section_info(which, L)["bits"]
            assert ob.container_bits(w) == 16
            codes, exps = random_section(w, elo, ehi)
            s.import_section(which, L, w, codes.view(np.uint8), exps)
            secs[which] = pw.Codes(codes, exps, B, w)
        s.up_sweep(L, torch.from_numpy(e_np).cuda())
        ym, ye, yw = s.export_section("y", L)
        um, ue, uw = s.export_section("u", L)
    del f
    ym = ym.view(np.int16).reshape(n, n, n // B, B)
    ye = ye.reshape(n, n, n // B)
    um = um.view(np.int16).reshape(n, n, n // B, B)
    ue = ue.reshape(n, n, n // B)
    rows = [(0, 3, 0), (1, 1, 0), (n - 1, n - 1, n // B - 1), (2, n - 1, 3), (n - 1, 1, 5), (n // 2, 0, 7)]
    rows += [tuple(int(v) for v in r) for r in np.stack([rng.integers(0, n, 44), rng.integers(0, n, 44),
                                                         rng.integers(0, n // B, 44)], axis=1)]
    for z, y, bx in rows:
        my, ey, mu, eu = pw.up_sweep_block(secs["r"], secs["ypre"], secs["u"], e_np, L, nu, z, y, bx, B, yw, uw)
        assert int(ye[z, y, bx]) == ey and np.array_equal(ym[z, y, bx].astype(np.int64), my), (z, y, bx)
        assert int(ue[z, y, bx]) == eu and np.array_equal(um[z, y, bx].astype(np.int64), mu), (z, y, bx)
