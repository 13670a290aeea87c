"""Plain FMG with iterative refinement — oracle (test infrastructure only).

The comparator the compact method is measured against: full multigrid that
keeps the standard representation, iterating on the residual equation on
every FMG level (supplement, Alg. SM2, "FMG using IR on each level") with
the correction-scheme V-cycle of the supplement (Sec. SM1.1.1): pre-smooth,
restrict the residual, recurse, prolongate and add the coarse correction,
post-smooth; exact solve on the coarsest level.
"""
from __future__ import annotations

import numpy as np

from .grid import coarse_solve, hierarchy, inject, prolong, restrict, smooth, to_full


def cs_vcycle(ops, level, r, cfg, T):
    """Correction-scheme V(nu1, nu2) cycle for ``A y = r`` from ``y = 0``."""
    lc = cfg.coarsest
    if level == lc:
        return coarse_solve(ops[lc], r).astype(T)
    lv = ops[level]
    r = np.asarray(r, dtype=T)
    y = smooth(lv, np.zeros_like(r), r, cfg.nu_pre, cfg.smoother, cfg.omega, T)
    rc = restrict(r - lv.apply(y, T), T)
    ec = cs_vcycle(ops, level - 1, rc, cfg, T)
    y = y + prolong(ec, T)
    return smooth(lv, y, r, cfg.nu_post, cfg.smoother, cfg.omega, T)


def fmg_solve(f_full: np.ndarray, cfg, kappa=None, history=None, vcycle_dtype=np.float64):
    """Alg. SM2 in float64 storage; the V-cycle runs in ``vcycle_dtype``.

    ``cfg`` is an :class:`oracle.compact.Config` (its width fields are
    ignored).  Returns the solution on the ``(2**L + 1)**dim`` node grid.
    """
    lc, L = cfg.coarsest, cfg.L
    ops = hierarchy(cfg.dim, L, lc, cfg.op, kappa)
    u = coarse_solve(ops[lc], inject(f_full, L, lc))
    for Lp in range(lc + 1, L + 1):
        u = prolong(u, np.float64)
        f_level = inject(f_full, L, Lp)
        iters = cfg.ir_iters + (cfg.final_iters if Lp == L else 0)
        for _ in range(iters):
            r = f_level - ops[Lp].apply(u, np.float64)
            if history is not None:
                history.append(float(np.linalg.norm(r)))
            y = cs_vcycle(ops, Lp, r, cfg, vcycle_dtype)
            u = u + y.astype(np.float64)
    return to_full(u)


def vcycles_to_convergence(f_full, cfg, kappa=None, rtol=1e-13, max_cycles=60):
    """Discrete solution ``u_h`` by FP64 V-cycles until the residual stagnates
    (the paper's reference-solution idea, Sec. 7.1, in float64)."""
    L, lc = cfg.L, cfg.coarsest
    ops = hierarchy(cfg.dim, L, lc, cfg.op, kappa)
    f = inject(f_full, L, L)
    fn = np.linalg.norm(f)
    u = np.zeros_like(f)
    best = np.inf
    for _ in range(max_cycles):
        r = f - ops[L].apply(u, np.float64)
        rn = np.linalg.norm(r)
        if rn <= rtol * fn or rn >= 0.9 * best:
            break
        best = min(best, rn)
        u = u + cs_vcycle(ops, L, r, cfg, np.float64)
    return to_full(u)
