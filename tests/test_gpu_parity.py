"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

* BFP codec: bit-exact codes and exponents, exact decode, over widths,
  block sizes, ragged lengths and both input types;
* one IR residual (Alg. 2) on identical imported sections: bit-exact codes;
* one compact V-cycle plus correction on identical inputs against the
  oracle run in float32 (the GPU V-cycle precision): bit-exact sections;
* whole compact FMG, plain FP64 FMG, the V-cycle entry and the adjoint
  gradient against the oracle on small grids spanning many BFP blocks.
"""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import adjoint as oa
from oracle import bfp as ob
from oracle import compact as oc
from oracle import grid as og
from oracle import plain as op

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cmg(gpu_lib):
    import paper_2511_19036_amd
    return paper_2511_19036_amd


def _codes(codes_u8, w, count):
    return ob.unpack(np.ascontiguousarray(codes_u8).tobytes(), w, count)


# ------------------------------------------------------------------ codec
@pytest.mark.parametrize("n", [1, 63, 1000, 4097])
@pytest.mark.parametrize("w", [2, 3, 8, 11, 12, 16, 17, 24, 33, 53])
@pytest.mark.parametrize("B", [32, 64])
@pytest.mark.parametrize("f64", [True, False])
def test_codec_bit_exact(cmg, n, w, B, f64):
    rng = np.random.default_rng(n * 1000 + w * 10 + B)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
    x[::7] = 0.0                                # zero entries and (for small n) zero blocks
    if n > 200:
        x[128:192] = 0.0                        # an all-zero block
        x[200] = 2.5 * 2.0 ** -30               # tie cases scaled into a block
    if not f64:
        x = x.astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    codes, exps = cmg.bfp_encode(xt, B, w)
    m_ref, e_ref = ob.encode(x, B, w)
    nb = (n + B - 1) // B
    assert np.array_equal(exps.cpu().numpy()[:nb], e_ref)
    assert np.array_equal(_codes(codes.cpu().numpy(), w, nb * B), m_ref)
    dec = cmg.bfp_decode(codes, exps, n, B, w).cpu().numpy()
    assert np.array_equal(dec, ob.decode(m_ref, e_ref, B, w, n))


def test_codec_rejects_nonfinite(cmg):
    x = torch.zeros(100, dtype=torch.float64, device="cuda")
    x[17] = float("nan")
    with pytest.raises(cmg.CmgError) as ei:
        cmg.bfp_encode(x, 64, 8)
    assert ei.value.status == 5


# ------------------------------------------------------------ step parity
CFGS = {
    # L >= 6 runs the fused 3-D kernels on the fine levels, per-operation below
    "3d-L7-b16": dict(dim=3, L=7, smoother="rbgs", omega=1.0, block=64, bits=16),
    "3d-L7-b12-B32": dict(dim=3, L=7, smoother="rbgs", omega=1.0, block=32, bits=12),
    "3d-L7-b12": dict(dim=3, L=7, smoother="rbgs", omega=1.0, block=64, bits=12),
    "3d-L7-b8-nu1": dict(dim=3, L=7, smoother="rbgs", omega=1.0, block=64, bits=8, nu=1),
    "3d-L6-b10": dict(dim=3, L=6, smoother="rbgs", omega=1.0, block=64, bits=10),
    "3d-rbgs-b16": dict(dim=3, L=5, smoother="rbgs", omega=1.0, block=64, bits=16),
    "3d-rbgs-b8": dict(dim=3, L=5, smoother="rbgs", omega=1.0, block=64, bits=8),
    "3d-rbgs-b12": dict(dim=3, L=5, smoother="rbgs", omega=1.0, block=64, bits=12),
    "2d-wjacobi-b16": dict(dim=2, L=7, smoother="wjacobi", omega=0.8, block=32, bits=16),
    "2d-wjacobi-b11": dict(dim=2, L=6, smoother="wjacobi", omega=0.8, block=32, bits=11),
    # the paper's own cycle, V(0,1) Gauss-Seidel (no pre-smoothing: y' = 0 on the way down)
    "3d-L7-V01-b12": dict(dim=3, L=7, smoother="rbgs", omega=1.0, block=64, bits=12, nu_pre=0, nu_post=1),
    "2d-L6-V01-b16": dict(dim=2, L=6, smoother="rbgs", omega=1.0, block=32, bits=16, nu_pre=0, nu_post=1),
}


def _nus(c):
    nu = c.get("nu", 2)
    return c.get("nu_pre", nu), c.get("nu_post", nu)


def _oracle_cfg(c, **kw):
    n1, n2 = _nus(c)
    return oc.Config(dim=c["dim"], L=c["L"], smoother=c["smoother"], omega=c["omega"], block=c["block"],
                     bits_u=c["bits"], bits_r=c["bits"], bits_y=c["bits"], nu_pre=n1, nu_post=n2, **kw)


def _solver(cmg, c, **kw):
    n1, n2 = _nus(c)
    return cmg.Solver(c["dim"], c["L"], smoother=c["smoother"], omega=c["omega"], bfp_block=c["block"],
                      bits=c["bits"], nu_pre=n1, nu_post=n2, **kw)


def _random_sections(cfg, Lp, seed):
    rng = np.random.default_rng(seed)
    U = {}
    for level in range(cfg.coarsest, Lp + 1):
        n = 1 << level
        x = np.zeros((n,) * cfg.dim)
        x[(slice(1, None),) * cfg.dim] = rng.standard_normal((n - 1,) * cfg.dim) * 2.0 ** (-2 * level)
        U[level] = oc.Section.quantize(x, cfg.block, cfg.w_u(level, Lp))
    return U


def _enter_all(s, L, f):
    for level in range(1, L + 1):
        s.enter_level(level, f)


def _export(s, which, level):
    codes, exps, bits = s.export_section(which, level)
    nb = exps.size
    return _codes(codes, bits, nb * s.opts.bfp_block), exps, bits


@pytest.mark.parametrize("name", list(CFGS))
def test_ir_residual_bit_exact(cmg, name):
    c = CFGS[name]
    cfg = _oracle_cfg(c)
    L = c["L"]
    f_np = S.gaussian_noise_rhs(c["dim"], L, sigma=0.1, seed=1)
    f = torch.from_numpy(f_np).cuda()
    U = _random_sections(cfg, L, 5)
    with _solver(cmg, c) as s:
        _enter_all(s, L, f)
        for level, sec in U.items():
            s.import_section("u", level, sec.w, np.frombuffer(ob.pack(sec.m, sec.w), dtype=np.uint8), sec.e)
        s.ir_residual(f)
        ops = og.hierarchy(c["dim"], L, 1)
        # without pre-smoothing every level's residual comes from Alg. 2's chain
        R = oc.residual_hierarchy(U, og.inject(f_np, L, L), ops, cfg, L)
        got = {level: _export(s, "r", level) for level in R}
    assert sorted(R) == (list(range(1, L + 1)) if _nus(c)[0] == 0 else [L])
    for level, g in R.items():
        m, e, bits = got[level]
        assert bits == g.w, level
        assert np.array_equal(e, g.e), level
        assert np.array_equal(m, g.m), level


@pytest.mark.parametrize("name", list(CFGS))
def test_vcycle_step_bit_exact(cmg, name):
    c = CFGS[name]
    cfg = _oracle_cfg(c)
    L = c["L"]
    f_np = S.gaussian_noise_rhs(c["dim"], L, sigma=0.1, seed=2)
    f = torch.from_numpy(f_np).cuda()
    U = _random_sections(cfg, L, 7)
    got = {}
    for keep in (True, False):
        with _solver(cmg, c, keep_correction=keep) as s:
            _enter_all(s, L, f)
            for level, sec in U.items():
                s.import_section("u", level, sec.w, np.frombuffer(ob.pack(sec.m, sec.w), dtype=np.uint8), sec.e)
            s.ir_residual(f)
            s.vcycle_correct()
            kinds = ("u", "y", "r") if keep else ("u", "r")
            got[keep] = {(w, level): _export(s, w, level) for w in kinds for level in range(1, L + 1)}
            if not keep:  # the correction is not kept: its export is refused
                with pytest.raises(cmg.CmgError) as ei:
                    s.export_section("y", L)
                assert ei.value.status == 2
    # without the kept correction sections the solution and residuals are the same bits
    for key, (m, e, bits) in got[False].items():
        m1, e1, bits1 = got[True][key]
        assert bits == bits1 and np.array_equal(e, e1) and np.array_equal(m, m1), key
    got = got[True]
    ops = og.hierarchy(c["dim"], L, 1)
    g = oc.residual_hierarchy(U, og.inject(f_np, L, L), ops, cfg, L)
    trace = {}
    Y = oc.vcycle_correct(U, g, ops, cfg, L, trace=trace)
    for level in range(1, L + 1):
        for which, sec in (("u", U[level]), ("y", Y[level]), ("r", trace["G"][level])):
            m, e, bits = got[(which, level)]
            assert bits == sec.w, (which, level)
            assert np.array_equal(e, sec.e), (which, level)
            assert np.array_equal(m, sec.m), (which, level)


# ------------------------------------------------------------ whole solves
@pytest.mark.parametrize("name", list(CFGS))
def test_compact_fmg_matches_oracle(cmg, name):
    c = CFGS[name]
    cfg = _oracle_cfg(c)
    L = c["L"]
    f_np = S.gaussian_noise_rhs(c["dim"], L, sigma=1e-3, seed=0)
    with _solver(cmg, c) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
        secs = {level: _export(s, "u", level) for level in range(1, L + 1)}
    u_ref, U = oc.fmg_solve(f_np, cfg)
    for level in range(1, L + 1):
        m, e, bits = secs[level]
        assert bits == U[level].w
        assert np.array_equal(e, U[level].e) and np.array_equal(m, U[level].m), level
    assert np.array_equal(u, u_ref)


@pytest.mark.parametrize("dim,L,smoother,omega", [(2, 6, "wjacobi", 0.8), (3, 5, "rbgs", 1.0), (3, 7, "rbgs", 1.0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plain_fmg_matches_oracle(cmg, dim, L, smoother, omega, prec):
    f_np = S.gaussian_noise_rhs(dim, L, sigma=1e-3, seed=3)
    cfg = oc.Config(dim=dim, L=L, smoother=smoother, omega=omega)
    T = np.float64 if prec == "fp64" else np.float32
    with cmg.Solver(dim, L, smoother=smoother, omega=omega, storage="plain", vcycle_prec=prec) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
    u_ref = op.fmg_solve(f_np, cfg, vcycle_dtype=T)
    assert np.array_equal(u, u_ref)


@pytest.mark.parametrize("name", ["3d-rbgs-b16", "2d-wjacobi-b16", "3d-L7-b16", "3d-L7-V01-b12", "2d-L6-V01-b16"])
def test_vcycle_entry_matches_oracle(cmg, name):
    c = CFGS[name]
    cfg = _oracle_cfg(c)
    r_np = S.gaussian_noise_rhs(c["dim"], c["L"], sigma=1.0, seed=9)
    with _solver(cmg, c) as s:
        y = s.vcycle(torch.from_numpy(r_np).cuda()[None])[0].cpu().numpy()
    assert np.array_equal(y, oc.vcycle_standard(r_np, cfg))


# 3-D L = 4 runs in the single-workgroup V-cycle; L >= 6 also runs the
# one-launch sweeps and the fused per-operation kernels of levels 5 and up.
@pytest.mark.parametrize("dim,L,smoother,omega,block",
                         [(3, 4, "rbgs", 1.0, 64), (2, 5, "wjacobi", 0.8, 32), (3, 6, "rbgs", 1.0, 64),
                          (3, 7, "rbgs", 1.0, 32)])
def test_diffusion_fmg_and_gradient_match_oracle(cmg, dim, L, smoother, omega, block):
    kappa = S.lognormal_kappa(dim, L, 0.2, 1)
    kobs = S.lognormal_kappa(dim, L, 0.2, 2)
    f_np = np.zeros(((1 << L) + 1,) * dim)
    f_np[(slice(1, -1),) * dim] = 1.0
    cfg = oc.Config(dim=dim, L=L, op="diffusion", smoother=smoother, omega=omega, block=block)
    u_ref, _ = oc.fmg_solve(f_np, cfg, kappa)
    uobs, _ = oc.fmg_solve(f_np, cfg, kobs)
    dj = oa.loss_grad_u(u_ref, uobs)
    lam_ref, _ = oc.fmg_solve(dj, cfg, kappa)
    g_ref = oa.grad_kappa(u_ref, lam_ref)
    kt = torch.from_numpy(kappa).cuda()
    with cmg.Solver(dim, L, op="diffusion", kappa=kt, smoother=smoother, omega=omega, bfp_block=block) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])
        assert np.array_equal(u[0].cpu().numpy(), u_ref)
        lam, g = s.adjoint(u, torch.from_numpy(dj).cuda()[None])
    assert np.array_equal(lam[0].cpu().numpy(), lam_ref)
    assert np.array_equal(g.cpu().numpy(), g_ref)


@pytest.mark.parametrize("op_,nu", [("diffusion", 1), ("poisson", 1), ("poisson", 2)])
def test_per_operation_fmg_matches_oracle(cmg, op_, nu):
    """Compact FMG on the per-operation kernels at 65^3: diffusion, or Poisson
    with the float64 V-cycle (no fused level kernels), V(nu, nu); nu = 1 ends
    a smoothing with its one-launch sweep in the scratch array."""
    dim, L = 3, 6
    f_np = S.gaussian_noise_rhs(dim, L, sigma=1e-3, seed=4)
    kw = dict(op=op_)
    if op_ == "diffusion":
        kappa = S.lognormal_kappa(dim, L, 0.2, 3)
        cfg = oc.Config(dim=dim, L=L, op=op_, nu_pre=nu, nu_post=nu)
        u_ref, _ = oc.fmg_solve(f_np, cfg, kappa)
        kw.update(kappa=torch.from_numpy(kappa).cuda())
    else:
        cfg = oc.Config(dim=dim, L=L, nu_pre=nu, nu_post=nu, vcycle_dtype=np.float64)
        u_ref, _ = oc.fmg_solve(f_np, cfg)
        kw.update(vcycle_prec="fp64")
    with cmg.Solver(dim, L, smoother="rbgs", bfp_block=64, bits=16, nu_pre=nu, nu_post=nu, **kw) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
    assert np.array_equal(u, u_ref)


def test_residual_norms_recorded(cmg):
    dim, L = 3, 7
    f_np = S.sine_rhs(dim, L)
    hist = []
    cfg = oc.Config(dim=dim, L=L, bits_u=16, bits_r=16, bits_y=16)
    oc.fmg_solve(f_np, cfg, history=hist)
    with cmg.Solver(dim, L, bits=16) as s:
        _, norms = s.solve(torch.from_numpy(f_np).cuda()[None], record=True)
    assert len(norms) == len(hist) == 2 * (L - 1)
    assert np.allclose(norms, hist, rtol=1e-10)


def test_nonfinite_rhs_reported(cmg):
    f = torch.zeros((1, 65, 65, 65), dtype=torch.float64, device="cuda")
    f[0, 30, 30, 30] = float("inf")
    with cmg.Solver(3, 6, bits=16) as s:
        with pytest.raises(cmg.CmgError) as ei:
            s.solve(f)
        assert ei.value.status == 5
        ok = s.solve(torch.zeros_like(f))          # the context stays usable
        assert float(ok.abs().max()) == 0.0


# ------------------------------------------------------------ accuracy
@pytest.mark.parametrize("bits", [8, 12, 16])
def test_gpu_fmg_discretisation_accuracy_3d(cmg, bits):
    dim, L = 3, 7
    h = 2.0 ** -L
    us = S.sine_solution(dim, L)
    uh = ((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2 * us
    with cmg.Solver(dim, L, smoother="rbgs", bits=bits) as s:
        u = s.solve(torch.from_numpy(S.sine_rhs(dim, L)).cuda()[None])[0].cpu().numpy()
    disc = og.norm_h(uh - us, h)
    assert og.norm_h(u - us, h) <= 2.0 * disc
    assert og.norm_h(u - uh, h) <= 0.5 * disc


# ------------------------------------------------------ coarsest level 2
@pytest.mark.parametrize("name", ["3d-rbgs-b12", "3d-L7-b16", "2d-wjacobi-b16", "3d-L7-V01-b12"])
def test_coarsest_level_two_matches_oracle(cmg, name):
    """A coarsest level of 3^dim interior nodes solved by the dense L D L^T
    factorisation: the whole compact FMG (single-workgroup V-cycle, fused
    and per-operation levels) and the plain FP64 FMG, bit for bit."""
    c = CFGS[name]
    cfg = _oracle_cfg(c, coarsest=2)
    L = c["L"]
    f_np = S.gaussian_noise_rhs(c["dim"], L, sigma=1e-3, seed=6)
    with _solver(cmg, c, coarsest=2) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
    u_ref, _ = oc.fmg_solve(f_np, cfg)
    assert np.array_equal(u, u_ref)
    with _solver(cmg, c, coarsest=2, storage="plain", vcycle_prec="fp64") as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
    assert np.array_equal(u, op.fmg_solve(f_np, cfg, vcycle_dtype=np.float64))


def test_coarsest_level_two_diffusion_matches_oracle(cmg):
    dim, L = 3, 5
    kappa = S.lognormal_kappa(dim, L, 0.2, 1)
    f_np = np.zeros(((1 << L) + 1,) * dim)
    f_np[(slice(1, -1),) * dim] = 1.0
    cfg = oc.Config(dim=dim, L=L, coarsest=2, op="diffusion")
    with cmg.Solver(dim, L, op="diffusion", coarsest=2, kappa=torch.from_numpy(kappa).cuda()) as s:
        u = s.solve(torch.from_numpy(f_np).cuda()[None])[0].cpu().numpy()
    u_ref, _ = oc.fmg_solve(f_np, cfg, kappa)
    assert np.array_equal(u, u_ref)


@pytest.mark.parametrize("storage", ["compact", "plain"])
def test_divergence_reported(cmg, storage):
    """Weighted Jacobi with omega = 1.99 amplifies the highest grid mode by
    |1 - 2 omega| ~ 3 per sweep: the IR residual grows from one iteration to
    the next and the solve ends with CMG_ERR_NOT_CONVERGED (the kernels run
    normally; only the host reads the monitor).  omega = 0.8 on the same
    problem converges and reports nothing."""
    f = torch.from_numpy(S.gaussian_noise_rhs(2, 5, sigma=1.0, seed=8)).cuda()[None]
    kw = dict(smoother="wjacobi", bfp_block=32, bits=16, storage=storage)
    with cmg.Solver(2, 5, omega=1.99, **kw) as s:
        with pytest.raises(cmg.CmgError) as ei:
            s.solve(f)
        assert ei.value.status == 6
        assert "FMG level" in str(ei.value)
    with cmg.Solver(2, 5, omega=0.8, **kw) as s:
        _, norms = s.solve(f, record=True)
    assert all(b < a for a, b in zip(norms[0::2], norms[1::2]))


def test_new_level_solution_reads_as_zero(cmg):
    """A new FMG level's u' is zero.  On the fused 3-D levels its zero fill
    is left to the first reader that needs it, and the coarser sections
    take the level's widths at their first correction: decoding the
    solution, or exporting the sections, right after entering the level
    gives the oracle's decode of the coarser sections with a zero finest
    section, the zero section itself and the widened coarser ones."""
    c = CFGS["3d-L7-b16"]
    cfg = _oracle_cfg(c)
    L = c["L"]
    f = torch.from_numpy(S.gaussian_noise_rhs(3, L, sigma=0.1, seed=2)).cuda()
    with _solver(cmg, c) as s:
        for level in range(1, L + 1):
            s.enter_level(level, f)
            if 1 < level < L:  # the coarsest level is solved on entry
                s.ir_residual(f)
                s.vcycle_correct()
        u_dec = s.decode_solution(L).cpu().numpy()
        secs = {level: _export(s, "u", level) for level in range(1, L + 1)}
    m, e, bits = secs[L]
    assert bits == cfg.w_u(L, L) and not np.any(m)
    # the coarser sections come out at this level's widths (Table 1), their
    # codes widened on export: the same values
    assert all(w == cfg.w_u(level, L) for level, (_, _, w) in secs.items())
    U = {level: oc.Section(3, level, cfg.block, w, m=mm.astype(np.int64), e=ee.astype(np.int64))
         for level, (mm, ee, w) in secs.items()}
    ref = oc.decode_chain(U, 1, L)
    n = 1 << L
    assert np.any(ref)
    assert np.array_equal(u_dec[:n, :n, :n], ref)
    assert not np.any(u_dec[n]) and not np.any(u_dec[:, n]) and not np.any(u_dec[:, :, n])
