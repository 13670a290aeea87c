"""Pins of the oracle's multigrid algorithms (no GPU).

* closed-form discrete solution of the sine problem and the paper's
  acceptance criteria (Sec. 7.1, eqs. experiment-successful and -order);
* the compact cycle from a zero guess equals the correction-scheme V-cycle
  (derived from eq. cfas: with ``y' = 0``, ``r - s`` is the restricted
  residual and ``z`` is the prolongated coarse correction);
* the decode identity (eq. compact-to-standard) against dense products;
* V-cycle contraction against a two-grid bound from dense matrices;
* dense direct solves for noisy right-hand sides;
* storage of regressive-precision vectors against Sec. 6.1.1.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import bfp, compact, dense, grid, plain
from oracle import pointwise as pw


def _closed_form(dim, L):
    h = 2.0 ** -L
    us = S.sine_solution(dim, L)
    ch = ((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2
    return us, ch * us, h


def test_closed_form_discrete_solution():
    # A u_h = f exactly for the sine right-hand side
    for dim, L in [(2, 5), (3, 4)]:
        us, uh, h = _closed_form(dim, L)
        f = S.sine_rhs(dim, L)
        lv = grid.Level(dim, L)
        n = 1 << L
        r = grid.inject(f, L, L) - lv.apply(uh[(slice(0, n),) * dim], np.float64)
        assert np.abs(r).max() < 1e-11 * np.abs(f).max()
    # relative discretisation error c_h - 1 at h = 1/128
    h = 1.0 / 128
    assert abs(((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2 - 1 - 5.020e-5) < 1e-8


CASES = [
    dict(dim=2, smoother="wjacobi", omega=0.8, block=32, Ls=(4, 5, 6), bits=12),
    dict(dim=2, smoother="wjacobi", omega=0.8, block=32, Ls=(4, 5, 6), bits=16),
    dict(dim=3, smoother="rbgs", omega=1.0, block=64, Ls=(3, 4, 5), bits=8),
    dict(dim=3, smoother="rbgs", omega=1.0, block=64, Ls=(3, 4, 5), bits=16),
]


@pytest.mark.parametrize("case", CASES, ids=["2d-b12", "2d-b16", "3d-b8", "3d-b16"])
def test_compact_fmg_reaches_discretisation_accuracy(case):
    # like the paper (Sec. 7.1) the finest widths are chosen per problem
    bits = case["bits"]
    errs = []
    for L in case["Ls"]:
        us, uh, h = _closed_form(case["dim"], L)
        cfg = compact.Config(dim=case["dim"], L=L, smoother=case["smoother"], omega=case["omega"],
                             block=case["block"], bits_u=bits, bits_r=bits, bits_y=bits)
        u, _ = compact.fmg_solve(S.sine_rhs(case["dim"], L), cfg)
        disc = grid.norm_h(uh - us, h)
        err = grid.norm_h(u - us, h)
        assert err <= 2.0 * disc                             # eq. experiment-successful
        assert grid.norm_h(u - uh, h) <= 0.5 * disc
        errs.append(err)
    for a, b in zip(errs, errs[1:]):
        assert -np.log2(b / a) >= 2.0 - 0.05                # eq. experiment-successful-order


@pytest.mark.parametrize("dim,smoother,omega,op", [
    (2, "wjacobi", 0.8, "poisson"), (3, "rbgs", 1.0, "poisson"), (3, "rbgs", 1.0, "diffusion")])
def test_unquantised_compact_fmg_equals_plain_fmg(dim, smoother, omega, op):
    L = 5 if dim == 2 else 4
    kappa = S.lognormal_kappa(dim, L, 0.2, 1) if op == "diffusion" else None
    f = S.gaussian_noise_rhs(dim, L, sigma=0.1, seed=4)
    base = dict(dim=dim, L=L, op=op, smoother=smoother, omega=omega, vcycle_dtype=np.float64)
    u_c, _ = compact.fmg_solve(f, compact.Config(quantize=False, **base), kappa)
    u_p = plain.fmg_solve(f, compact.Config(**base), kappa)
    assert np.abs(u_c - u_p).max() <= 1e-12 * np.abs(u_p).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_compact_vcycle_equals_correction_scheme(dim):
    L = 5 if dim == 2 else 4
    sm = "wjacobi" if dim == 2 else "rbgs"
    om = 0.8 if dim == 2 else 1.0
    cfg = compact.Config(dim=dim, L=L, smoother=sm, omega=om, quantize=False, vcycle_dtype=np.float64)
    r = S.gaussian_noise_rhs(dim, L, sigma=1.0, seed=8)
    y_c = compact.vcycle_standard(r, cfg)
    ops = grid.hierarchy(dim, L, 1)
    y_p = plain.cs_vcycle(ops, L, grid.inject(r, L, L), cfg, np.float64)
    assert np.abs(y_c[(slice(0, 1 << L),) * dim] - y_p).max() <= 1e-13 * np.abs(y_p).max()


def test_decode_identity_against_dense_products():
    dim, L, lc = 2, 4, 1
    rng = np.random.default_rng(3)
    U = {}
    for level in range(lc, L + 1):
        n = 1 << level
        x = np.zeros((n,) * dim)
        x[1:, 1:] = rng.standard_normal((n - 1,) * dim) * 2.0 ** (-2 * level)
        U[level] = compact.Section.quantize(x, 32, 12)
    got = compact.decode_chain(U, lc, L)[1:, 1:].reshape(-1)
    expect = np.zeros(((1 << L) - 1) ** dim)
    for level in range(lc, L + 1):
        v = U[level].value()[1:, 1:].reshape(-1)
        for k in range(level + 1, L + 1):
            v = dense.prolongation(dim, k) @ v
        expect += v
    assert np.allclose(got, expect, rtol=1e-14, atol=1e-16)


def _dense_smoother(A, smoother, omega, dim, level):
    m = A.shape[0]
    if smoother == "wjacobi":
        return np.eye(m) - omega * A / np.diag(A)[:, None]
    import itertools
    n = 1 << level
    nodes = list(itertools.product(range(1, n), repeat=dim))
    order = [i for i, p in enumerate(nodes) if sum(p) % 2 == 0] + \
            [i for i, p in enumerate(nodes) if sum(p) % 2 == 1]
    Pm = np.eye(m)[order]
    Ap = Pm @ A @ Pm.T
    Sp = np.eye(m) - np.linalg.solve(np.tril(Ap), Ap)
    return Pm.T @ Sp @ Pm


def _dense_vcycle_error(dim, L, lc, smoother, omega, nu1=2, nu2=2):
    """Error propagation ``I - M_L A_L`` of the V(nu1, nu2) cycle, built
    recursively from dense matrices: ``E_lc = 0`` (exact coarse solve) and
    ``E_l = S^nu2 (I - P (I - E_{l-1}) A_{l-1}^-1 R A_l) S^nu1``."""
    E = None
    for level in range(lc, L + 1):
        A = dense.poisson(dim, level)
        m = A.shape[0]
        if level == lc:
            E = np.zeros((m, m))
            continue
        Ac = dense.poisson(dim, level - 1)
        P = dense.prolongation(dim, level)
        R = (0.5 ** dim) * P.T
        Sm = _dense_smoother(A, smoother, omega, dim, level)
        Mc = (np.eye(Ac.shape[0]) - E) @ np.linalg.inv(Ac)
        E = np.linalg.matrix_power(Sm, nu2) @ (np.eye(m) - P @ Mc @ R @ A) @ \
            np.linalg.matrix_power(Sm, nu1)
    return E


@pytest.mark.parametrize("dim,L,smoother,omega,nu1,nu2", [
    (2, 5, "wjacobi", 0.8, 2, 2), (3, 3, "rbgs", 1.0, 2, 2),
    # the paper's own cycle: V(0,1) Gauss-Seidel (Alg. 1)
    (2, 4, "rbgs", 1.0, 0, 1), (3, 3, "rbgs", 1.0, 0, 1)])
def test_vcycle_error_map_equals_dense_recursion(dim, L, smoother, omega, nu1, nu2):
    E = _dense_vcycle_error(dim, L, 1, smoother, omega, nu1, nu2)
    cfg = compact.Config(dim=dim, L=L, smoother=smoother, omega=omega, quantize=False,
                         vcycle_dtype=np.float64, nu_pre=nu1, nu_post=nu2)
    n = 1 << L
    e = np.zeros((n + 1,) * dim)
    e[(slice(1, -1),) * dim] = np.random.default_rng(4).standard_normal((n - 1,) * dim)
    r = grid.to_full(grid.Level(dim, L).apply(e[(slice(0, n),) * dim], np.float64))
    e_new = (e - compact.vcycle_standard(r, cfg))[(slice(1, -1),) * dim].reshape(-1)
    ref = E @ e[(slice(1, -1),) * dim].reshape(-1)
    assert np.abs(e_new - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim,L,smoother,omega", [(2, 5, "wjacobi", 0.8), (3, 4, "rbgs", 1.0)])
def test_vcycle_contraction_within_two_grid_bound(dim, L, smoother, omega):
    A = dense.poisson(dim, L)
    Ac = dense.poisson(dim, L - 1)
    P = dense.prolongation(dim, L)
    R = (0.5 ** dim) * P.T
    Sm = _dense_smoother(A, smoother, omega, dim, L)
    S2 = Sm @ Sm
    E = S2 @ (np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, R @ A)) @ S2
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    for _ in range(200):
        x = E @ x
        nx = np.linalg.norm(x)
        x /= nx
    rho_tg = nx
    # V-cycle error contraction of the compact cycle (unquantised, float64)
    cfg = compact.Config(dim=dim, L=L, smoother=smoother, omega=omega, quantize=False,
                         vcycle_dtype=np.float64)
    n = 1 << L
    e = np.zeros((n + 1,) * dim)
    e[(slice(1, -1),) * dim] = np.random.default_rng(1).standard_normal((n - 1,) * dim)
    lv = grid.Level(dim, L)
    ratio = None
    for _ in range(25):
        r = grid.to_full(lv.apply(e[(slice(0, n),) * dim], np.float64))
        e_new = e - compact.vcycle_standard(r, cfg)
        ratio = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    # the multilevel cycle contracts nearly as well as the two-grid method
    assert ratio <= 1.5 * rho_tg
    assert ratio < 0.25


def test_noisy_rhs_against_dense_solve():
    dim, L = 2, 5
    f = S.gaussian_noise_rhs(dim, L, sigma=1e-3, seed=0)
    A = dense.poisson(dim, L)
    uh = np.zeros_like(f)
    uh[1:-1, 1:-1] = np.linalg.solve(A, f[1:-1, 1:-1].reshape(-1)).reshape((31, 31))
    cfg = compact.Config(dim=2, L=L, smoother="wjacobi", omega=0.8, block=32)
    u, _ = compact.fmg_solve(f, cfg)
    us, uh_sine, h = _closed_form(dim, L)
    disc = grid.norm_h(uh_sine - us, h)
    assert grid.norm_h(u - uh, h) <= 0.5 * disc
    # and the plain FMG agrees with the dense solve to the same accuracy
    up = plain.fmg_solve(f, cfg)
    assert grid.norm_h(up - uh, h) <= 0.5 * disc
    # converged V-cycles reach the dense solution
    uc = plain.vcycles_to_convergence(f, cfg)
    assert np.abs(uc - uh).max() <= 1e-12 * np.abs(uh).max()


@pytest.mark.parametrize("dim,b,k", [(3, 16, 1), (3, 8, 2), (2, 16, 1), (2, 5, 2)])
def test_regressive_storage_bound(dim, b, k):
    # Sec. 6.1.1: sum_l (k (L - l) + b) n_l < (2^d/(2^d-1) b + 2^d/(2^d-1)^2 k) n_L
    L = 10 if dim == 3 else 14
    cfg = compact.Config(dim=dim, L=L, bits_u=b, bits_r=b, bits_y=b, inc_u=k, inc_ry=k,
                         vcycle_dtype=np.float64)
    bits = compact.storage_bits(cfg)
    nL = (1 << L) ** dim
    c = 2 ** dim / (2 ** dim - 1)
    bound = (c * b + c / (2 ** dim - 1) * k) * nL
    assert bits["u"] < bound
    assert bits["u"] > 0.99 * bound


def test_width_schedule():
    cfg = compact.Config(dim=3, L=10, bits_u=16, bits_r=8, bits_y=8)
    assert cfg.w_u(10, 10) == 16 and cfg.w_u(1, 10) == 34
    assert cfg.w_r(10, 10) == 8 and cfg.w_r(1, 10) == 17
    cfg16 = compact.Config(dim=3, L=10)
    assert cfg16.w_r(1, 10) == 24                       # FP32 V-cycle cap
    assert compact.Config(dim=3, L=10, vcycle_dtype=np.float64).w_r(1, 10) == 25
    assert bfp.container_bits(cfg.w_u(1, 10)) == 64


# ------------------------------------------------- node-by-node residual
def _section_codes(sec):
    dt = {8: np.int8, 16: np.int16, 32: np.int32, 64: np.int64}[bfp.container_bits(sec.w)]
    return pw.Codes(sec.m.astype(dt), sec.e, sec.block, sec.w)


def _random_compact(L, bits, seed):
    cfg = compact.Config(dim=3, L=L, bits_u=bits, bits_r=bits, bits_y=bits)
    rng = np.random.default_rng(seed)
    U = {}
    for level in range(1, L + 1):
        n = 1 << level
        x = np.zeros((n,) * 3)
        x[1:, 1:, 1:] = rng.standard_normal((n - 1,) * 3) * 2.0 ** (-2 * level)
        U[level] = compact.Section.quantize(x, cfg.block, cfg.w_u(level, L))
    return cfg, U, rng


@pytest.mark.parametrize("L,bits", [(4, 16), (5, 17), (5, 30)])
def test_pointwise_decode_chain_equals_whole_array(L, bits):
    """The node-by-node decode chain (used at full size) equals the
    whole-array chain of eq. compact-to-standard at every node."""
    cfg, U, _ = _random_compact(L, bits, 100 * L + bits)
    n = 1 << L
    idx = np.stack(np.meshgrid(*[np.arange(n + 1)] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    got = pw.decode_chain_at({lv: _section_codes(s) for lv, s in U.items()}, 1, L, idx)
    assert np.array_equal(got.reshape((n + 1,) * 3), grid.to_full(compact.decode_chain(U, 1, L)))


def test_pointwise_residual_blocks_equal_whole_array():
    """Residual blocks of Alg. 2 evaluated node by node equal the
    whole-array residual section (64^3, sampled blocks incl. boundary rows)."""
    L = 6
    cfg, U, rng = _random_compact(L, 16, 7)
    n = 1 << L
    f = rng.standard_normal((n + 1,) * 3)
    g = compact.ir_residual(U, grid.inject(f, L, L), grid.hierarchy(3, L, 1), cfg, L)
    gm, ge = g.m.reshape(n, n, n), g.e.reshape(n, n)
    Uc = {lv: _section_codes(s) for lv, s in U.items()}
    rows = [(0, 5), (3, 0), (1, 1), (n - 1, n - 1)] + [tuple(r) for r in rng.integers(0, n, (12, 2))]
    for z, y in rows:
        m, e = pw.ir_residual_block(Uc, 1, L, f[z, y, :n], z, y, 0, cfg.block, cfg.w_r(L, L))
        assert np.array_equal(m, gm[z, y]) and e == int(ge[z, y]), (z, y)


def test_pointwise_down_sweep_and_restriction_equal_whole_array():
    """The node-local down sweep (y' = Q(S^nu(0; g))) and the residual
    restriction (g_{L-1} = Q(R(g - A y'))) equal the whole-array V-cycle's
    first level, traced, on sampled blocks of a 128^3 grid."""
    L, nu = 7, 2
    cfg = compact.Config(dim=3, L=L, bits_u=16, bits_r=16, bits_y=16, nu_pre=nu, nu_post=nu)
    rng = np.random.default_rng(3)
    n = 1 << L
    x = np.zeros((n,) * 3)
    x[1:, 1:, 1:] = rng.standard_normal((n - 1,) * 3)
    g = compact.Section.quantize(x, cfg.block, cfg.w_r(L, L))
    U = {lv: compact.Section.zeros(3, lv, cfg.block, cfg.w_u(lv, L)) for lv in range(1, L + 1)}
    trace = {}
    compact.vcycle_correct(U, g, grid.hierarchy(3, L, 1), cfg, L, trace=trace)
    yp, gc = trace["Ypre"][L], trace["G"][L - 1]
    G = _section_codes(g)
    m = n // 2
    rows = [(0, 3), (1, 1), (n - 1, n - 2), (5, n - 1)] + [tuple(r) for r in rng.integers(0, n, (8, 2))]
    for z, y in rows:
        for bx in range(n // cfg.block):
            mm, e = pw.down_sweep_block(G, L, nu, z, y, bx, cfg.block, cfg.w_y(L, L))
            k = (z * n + y) * n + bx * cfg.block
            assert np.array_equal(mm, yp.m[k:k + cfg.block]) and e == int(yp.e[k // cfg.block]), (z, y, bx)
    crow = [(0, 2), (1, 1), (m - 1, m - 1), (7, 0)] + [tuple(r) for r in rng.integers(0, m, (6, 2))]
    for K, J in crow:
        mm, e = pw.restrict_block(G, L, nu, K, J, 0, cfg.block, cfg.w_y(L, L), cfg.w_r(L - 1, L))
        k = (K * m + J) * m
        assert np.array_equal(mm, gc.m[k:k + cfg.block]) and e == int(gc.e[k // cfg.block]), (K, J)


# ------------------------------------------------ Alg. 2 restriction chain
@pytest.mark.parametrize("dim,L,w", [(2, 5, 6), (3, 4, 6), (3, 4, 12)])
def test_restrict_chain_against_dense_products(dim, L, w):
    # Alg. 2 restricts the unrounded t and rounds every level once:
    # r_l = fix(R_{l+1} ... R_L t).  With integer t every product and sum is
    # an exact dyadic rational, so the dense products R = 2^-d P^T applied
    # one after another give the exact values, and the codes must be equal.
    rng = np.random.default_rng(11)
    n = 1 << L
    t = np.zeros((n,) * dim)
    t[(slice(1, None),) * dim] = rng.integers(-1000, 1001, size=(n - 1,) * dim)
    B = 32 if dim == 2 else 64
    cfg = compact.Config(dim=dim, L=L, block=B, bits_r=w, nu_pre=0, nu_post=1)
    got = compact.restrict_chain(t, cfg, L, L)
    v = t[(slice(1, None),) * dim].reshape(-1)
    differs = 0
    for level in range(L, 0, -1):
        if level < L:
            v = (0.5 ** dim) * dense.prolongation(dim, level + 1).T @ v
        m = 1 << level
        x = np.zeros((m,) * dim)
        x[(slice(1, None),) * dim] = v.reshape((m - 1,) * dim)
        wl = cfg.w_r(level, L)
        codes, exps = bfp.encode(x.reshape(-1), B, wl)
        assert got[level].w == wl
        assert np.array_equal(got[level].e, exps) and np.array_equal(got[level].m, codes), level
        if level < L:
            # restricting the rounded finer level instead (the departure this
            # pin guards against) gives other codes at these widths
            rc = grid.restrict(got[level + 1].value(np.float64), np.float64)
            mc, _ = bfp.encode(rc.reshape(-1), B, wl)
            differs += int(np.count_nonzero(mc != codes))
    assert differs > 0


def test_residual_hierarchy_without_presmoothing():
    # V(0, nu2): the cycle takes every level's residual from Alg. 2; with
    # pre-smoothing only the finest one (the cycle restricts g - A y')
    dim, L = 3, 4
    f = S.gaussian_noise_rhs(dim, L, sigma=0.1, seed=2)
    ops = grid.hierarchy(dim, L, 1)
    for nu1, levels in ((0, list(range(1, L + 1))), (2, [L])):
        cfg = compact.Config(dim=dim, L=L, bits_u=10, bits_r=10, bits_y=10, nu_pre=nu1, nu_post=1)
        U = {lv: compact.Section.zeros(dim, lv, 64, cfg.w_u(lv, L)) for lv in range(1, L + 1)}
        R = compact.residual_hierarchy(U, grid.inject(f, L, L), ops, cfg, L)
        assert sorted(R) == levels
        chain = compact.restrict_chain(grid.inject(f, L, L), cfg, L, L)
        for lv in levels:
            assert np.array_equal(R[lv].m, chain[lv].m) and np.array_equal(R[lv].e, chain[lv].e)
    with pytest.raises(ValueError):
        cfg = compact.Config(dim=dim, L=L, nu_pre=0, nu_post=1)
        compact.vcycle_correct(U, R[L], ops, cfg, L)


@pytest.mark.parametrize("nu1", [0, 2])
def test_exact_s_reading_unquantised_equals_correction_scheme(nu1):
    # keeping s apart in float64 (Alg. 1's fine-to-coarse sweep) is the same
    # cycle as the correction scheme when nothing is rounded
    dim, L = 3, 4
    cfg = compact.Config(dim=dim, L=L, quantize=False, vcycle_dtype=np.float64, s_mode="fp64",
                         nu_pre=nu1, nu_post=2)
    r = S.gaussian_noise_rhs(dim, L, sigma=1.0, seed=9)
    y_c = compact.vcycle_standard(r, cfg)
    ops = grid.hierarchy(dim, L, 1)
    y_p = plain.cs_vcycle(ops, L, grid.inject(r, L, L), cfg, np.float64)
    assert np.abs(y_c[(slice(0, 1 << L),) * dim] - y_p).max() <= 1e-13 * np.abs(y_p).max()


@pytest.mark.parametrize("bits,tol", [(8, 0.15), (16, 0.01)])
def test_fold_reading_changes_the_solution_little(bits, tol):
    # The paper leaves the precision of s open (Sec. 4).  Storing g = r - s
    # at the residual width ("fold", the GPU's reading) against keeping r
    # from Alg. 2's chain and s unrounded in float64: both meet the
    # acceptance test, and the solutions differ by a small fraction of the
    # discretisation error (measured 0.08 / 0.005 / 0.0003 at 8 / 12 / 16
    # bits, 3-D L = 5).
    dim, L = 3, 5
    us, uh, h = _closed_form(dim, L)
    disc = grid.norm_h(uh - us, h)
    sols = {}
    for mode in ("fold", "fp64"):
        cfg = compact.Config(dim=dim, L=L, bits_u=bits, bits_r=bits, bits_y=bits, s_mode=mode)
        u, _ = compact.fmg_solve(S.sine_rhs(dim, L), cfg)
        assert grid.norm_h(u - us, h) <= 2.0 * disc
        assert grid.norm_h(u - uh, h) <= 0.5 * disc
        sols[mode] = u
    diff = grid.norm_h(sols["fold"] - sols["fp64"], h) / disc
    print(f"fold vs fp64 s at {bits} bits: |u_fold - u_fp64| / disc = {diff:.3e}")
    assert diff <= tol


# ------------------------------------------------ coarsest level 2
@pytest.mark.parametrize("dim,L", [(2, 6), (3, 5)])
def test_coarsest_level_two(dim, L):
    # a dense coarsest solve of 3^dim nodes instead of one: the unquantised
    # compact FMG still equals the plain FP64 FMG, and the quantised one
    # meets the acceptance test on the sine problem
    f = S.sine_rhs(dim, L)
    cfg = compact.Config(dim=dim, L=L, coarsest=2, quantize=False, vcycle_dtype=np.float64,
                         smoother="rbgs", omega=1.0)
    u_c, _ = compact.fmg_solve(f, cfg)
    u_p = plain.fmg_solve(f, cfg)
    assert np.abs(u_c - u_p).max() <= 1e-12 * np.abs(u_p).max()
    us, uh, h = _closed_form(dim, L)
    disc = grid.norm_h(uh - us, h)
    cfg = compact.Config(dim=dim, L=L, coarsest=2, bits_u=12, bits_r=12, bits_y=12)
    u, _ = compact.fmg_solve(f, cfg)
    assert grid.norm_h(u - us, h) <= 2.0 * disc
    assert grid.norm_h(u - uh, h) <= 0.5 * disc


@pytest.mark.parametrize("L", [6, 7])
def test_pointwise_up_sweep_equals_whole_array(L):
    """The node-local up sweep and correction (z = P e, y = S^nu(y'_pre;
    g - A z), y' = Q(y), u' = Q(u' + y')) equal the whole-array V-cycle's
    finest level, traced, on sampled blocks of 64^3 and 128^3 grids (random
    residual and solution sections; boundary rows included)."""
    nu = 2
    cfg = compact.Config(dim=3, L=L, bits_u=16, bits_r=16, bits_y=16, nu_pre=nu, nu_post=nu)
    rng = np.random.default_rng(30 + L)
    n = 1 << L
    x = np.zeros((n,) * 3)
    x[1:, 1:, 1:] = rng.standard_normal((n - 1,) * 3)
    g = compact.Section.quantize(x, cfg.block, cfg.w_r(L, L))
    U = {}
    for lv in range(1, L + 1):
        m = 1 << lv
        u = np.zeros((m,) * 3)
        u[1:, 1:, 1:] = rng.standard_normal((m - 1,) * 3) * 4.0 ** -lv
        U[lv] = compact.Section.quantize(u, cfg.block, cfg.w_u(lv, L))
    U0 = dict(U)
    trace = {}
    Y = compact.vcycle_correct(U, g, grid.hierarchy(3, L, 1), cfg, L, trace=trace)
    G, Yp = _section_codes(g), _section_codes(trace["Ypre"][L])
    Uc = _section_codes(U0[L])
    E = trace["E"][L - 1]
    assert E.dtype == np.float32 and E.shape == (n // 2,) * 3
    rows = [(0, 3), (1, 1), (n - 1, n - 2), (5, n - 1)] + [tuple(r) for r in rng.integers(0, n, (6, 2))]
    for z, y in rows:
        for bx in range(n // cfg.block):
            my, ey, mu, eu = pw.up_sweep_block(G, Yp, Uc, E, L, nu, z, y, bx, cfg.block, cfg.w_y(L, L),
                                               cfg.w_u(L, L))
            k = (z * n + y) * n + bx * cfg.block
            assert np.array_equal(my, Y[L].m[k:k + cfg.block]) and ey == int(Y[L].e[k // cfg.block]), (z, y, bx)
            assert np.array_equal(mu, U[L].m[k:k + cfg.block]) and eu == int(U[L].e[k // cfg.block]), (z, y, bx)
