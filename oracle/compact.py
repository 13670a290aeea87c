"""Compact full multigrid — oracle (test infrastructure only).

Follows the paper's algorithms step by step on whole-level numpy arrays:

* compact representation: ``u_L = u'_L + P_L (u'_{L-1} + ... + P_1 u'_0)``
  (Sec. 2, eq. compact-to-standard); sections in regressive precision
  ``k (L - l) + b`` bits on level ``l`` (Sec. 2.1, eq. regressive);
* residual: decode the standard representation level by level, form
  ``t = f - A u_L`` and round it to the residual precision; when the cycle
  has no pre-smoothing (V(0, nu2), the paper's own cycle) also restrict the
  unrounded ``t`` level by level in float64 and round each level once,
  ``r_l = fix(R_{l+1} ... R_L t)`` (Alg. 2, "restrict residual");
* V-cycle: the compact FAS cycle relaxes, on every level, eq. cfas
  ``A_l y'_l = r_l - s_l - A_l z_l`` (Sec. 3.2, Alg. 1).  With the initial
  guess ``y' = 0`` that IR guarantees (Sec. 4, nu = 1) and ``nu1`` pre- and
  ``nu2`` post-smoothing sweeps:

  - fine to coarse, ``g_l := r_l - s_l`` obeys
    ``g_{l-1} = R_l (g_l - A_l y'_l)`` where ``y'_l`` is the pre-smoothed
    (and stored, i.e. rounded) section: this is the recursion for ``s`` in
    Alg. 1 written for ``r - s``.  Without pre-smoothing ``y' = 0`` on the
    way down, so ``s = 0`` and ``g_l = r_l`` comes from Alg. 2's chain;
  - on the coarsest level the equation is solved exactly;
  - coarse to fine, ``z_l = P_l (y'_{l-1} + z_{l-1})`` (Alg. 1) and the
    post-smoother relaxes ``A_l y'_l = g_l - A_l z_l``;
  - the correction is added section by section, ``u'_l <- u'_l + y'_l``
    (Alg. 3, "apply correction"; Sec. 2.2 linear combinations);

* FMG: coarsest solve, then per level append a zero section and widen the
  others by ``k`` bits (Sec. 2.2, Alg. 3) and run ``N`` IR iterations.

Precision reading (Table 1 mapped to IEEE types): sections of ``u'`` carry
``b_u + k_u (L - l)`` bits (``k_u = p + 1 = 2``), residual and correction
``b + (L - l)`` bits (``k = m = 1``); the residual, decode chain, correction
and coarsest solve run in float64; the V-cycle arithmetic runs in
``vcycle_dtype`` (float32 by default), which caps residual/correction widths
at 24 bits (53 in float64).  The paper leaves the precision of ``s`` open
(Sec. 4); here ``g = r - s`` is stored at the residual's width
(``s_mode = "fold"``, what the GPU computes).  ``s_mode = "fp64"`` keeps
instead ``r_l`` from Alg. 2's chain and ``s_l`` unrounded in float64
(``s_{l-1} = R_l (A_l y'_l + s_l)``, Alg. 1's fine-to-coarse sweep) and
relaxes with ``r_l - s_l``: it measures what the fold reading changes when
``nu1 > 0`` (with ``nu1 = 0`` both modes are the same computation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bfp
from .grid import (coarse_solve, hierarchy, inject, prolong, restrict, smooth,
                   to_full)


@dataclass
class Config:
    dim: int
    L: int
    coarsest: int = 1
    op: str = "poisson"            # "poisson" | "diffusion"
    smoother: str = "rbgs"         # "rbgs" | "wjacobi"
    omega: float = 1.0
    nu_pre: int = 2
    nu_post: int = 2
    ir_iters: int = 2              # N, IR iterations per FMG level
    final_iters: int = 0           # extra IR iterations on the finest level
    block: int = 64
    bits_u: int = 16
    bits_r: int = 16
    bits_y: int = 16
    inc_u: int = 2
    inc_ry: int = 1
    vcycle_dtype: type = np.float32
    quantize: bool = True
    s_mode: str = "fold"           # "fold" | "fp64" (see the module docstring)

    def cap_ry(self) -> int:
        return 24 if self.vcycle_dtype == np.float32 else 53

    def w_u(self, level: int, Lp: int) -> int:
        return min(bfp.MAX_BITS, self.bits_u + self.inc_u * (Lp - level))

    def w_r(self, level: int, Lp: int) -> int:
        return min(self.cap_ry(), self.bits_r + self.inc_ry * (Lp - level))

    def w_y(self, level: int, Lp: int) -> int:
        return min(self.cap_ry(), self.bits_y + self.inc_ry * (Lp - level))


class Section:
    """One level of a compact vector: BFP codes, or raw float64 values when
    quantisation is switched off (used to check the cycle's algebra)."""

    def __init__(self, dim, level, block, w, m=None, e=None, raw=None):
        self.dim, self.level, self.block, self.w = dim, level, block, w
        self.n = 1 << level
        self.m, self.e, self.raw = m, e, raw

    @classmethod
    def quantize(cls, x: np.ndarray, block: int, w: int, on: bool = True):
        d, n = x.ndim, x.shape[0]
        level = n.bit_length() - 1
        if not on:
            return cls(d, level, block, w, raw=np.array(x, dtype=np.float64))
        m, e = bfp.encode(x.reshape(-1), block, w)
        return cls(d, level, block, w, m=m, e=e)

    @classmethod
    def zeros(cls, dim, level, block, w, on=True):
        return cls.quantize(np.zeros(((1 << level),) * dim), block, w, on)

    def value(self, T=np.float64) -> np.ndarray:
        shape = (self.n,) * self.dim
        if self.raw is not None:
            return self.raw.astype(T)
        size = self.n ** self.dim
        return bfp.decode(self.m, self.e, self.block, self.w, size, T).reshape(shape)

    def widen(self, w_new: int) -> "Section":
        k = w_new - self.w
        if k < 0:
            raise ValueError("widening cannot lower the width")
        if self.raw is not None:
            return Section(self.dim, self.level, self.block, w_new, raw=self.raw)
        return Section(self.dim, self.level, self.block, w_new, m=bfp.widen(self.m, k), e=self.e)


def decode_chain(U: dict, lc: int, Lp: int) -> np.ndarray:
    """Standard representation of the compact vector ``U`` on level ``Lp``
    (eq. compact-to-standard evaluated from the coarsest level up, Alg. 2)."""
    uh = U[lc].value(np.float64)
    for level in range(lc + 1, Lp + 1):
        uh = U[level].value(np.float64) + prolong(uh, np.float64)
    return uh


def restrict_chain(t: np.ndarray, cfg: Config, Lp: int, top: int) -> dict:
    """Alg. 2, "restrict residual": ``t_{l-1} = R_l t_l`` in float64 from the
    unrounded ``t`` of level ``top``, each level rounded once to its residual
    width, ``r_l = fix(t_l)``.  Returns ``{level: Section}`` for levels
    ``coarsest .. top``."""
    out = {top: Section.quantize(t, cfg.block, cfg.w_r(top, Lp), cfg.quantize)}
    for level in range(top - 1, cfg.coarsest - 1, -1):
        t = restrict(t, np.float64)
        out[level] = Section.quantize(t, cfg.block, cfg.w_r(level, Lp), cfg.quantize)
    return out


def chain_needed(cfg: Config) -> bool:
    """Whether the V-cycle takes the whole residual hierarchy from Alg. 2:
    without pre-smoothing (V(0, nu2)), or when ``s`` is kept separately."""
    return cfg.nu_pre == 0 or cfg.s_mode == "fp64"


def residual_hierarchy(U, f_level, ops, cfg: Config, Lp: int) -> dict:
    """Alg. 2 on FMG level ``Lp``: ``t = f - A u_Lp`` in float64 from the
    decoded solution, ``r_Lp = fix(t)``, and, when the V-cycle needs them,
    the restricted residuals of every coarser level.  Returns
    ``{level: Section}``."""
    uh = decode_chain(U, cfg.coarsest, Lp)
    t = f_level - ops[Lp].apply(uh, np.float64)
    if chain_needed(cfg):
        return restrict_chain(t, cfg, Lp, Lp)
    return {Lp: Section.quantize(t, cfg.block, cfg.w_r(Lp, Lp), cfg.quantize)}


def ir_residual(U, f_level, ops, cfg: Config, Lp: int) -> Section:
    """The finest section ``g_Lp = fix(f - A u_Lp)`` of Alg. 2 (float64)."""
    return residual_hierarchy(U, f_level, ops, cfg, Lp)[Lp]


def vcycle_correct(U, g_top, ops, cfg: Config, Lp: int, trace=None):
    """One compact V(nu1, nu2) cycle from a zero correction, then ``u' += y'``.

    ``g_top`` is the residual hierarchy of :func:`residual_hierarchy` (or
    its finest section alone, when the cycle restricts by itself).  Returns
    the correction sections ``Y`` (after post-smoothing).  If ``trace`` is a
    dict it receives the intermediate sections (``G``, the pre-smoothed
    ``Y``) and the coarse corrections ``E[l] = y'_l + z_l`` that enter the
    up sweep of level ``l + 1``, for inspection.
    """
    T = cfg.vcycle_dtype
    lc, B, on = cfg.coarsest, cfg.block, cfg.quantize
    R = dict(g_top) if isinstance(g_top, dict) else {Lp: g_top}
    exact_s = cfg.s_mode == "fp64"
    if cfg.s_mode not in ("fold", "fp64"):
        raise ValueError(cfg.s_mode)
    if chain_needed(cfg) and len(R) != Lp - lc + 1:
        raise ValueError("this cycle needs the residual of every level (Alg. 2)")
    G = {Lp: R[Lp]}
    s64 = {Lp: np.zeros((1 << Lp,) * cfg.dim)}            # s of the "fp64" reading
    Y = {}

    def rhs_of(level):                                     # r_l - s_l in the V-cycle type
        if exact_s:
            return (G[level].value(np.float64) - s64[level]).astype(T)
        return G[level].value(T)

    for level in range(Lp, lc, -1):                       # fine to coarse
        lv = ops[level]
        g = rhs_of(level)
        y = smooth(lv, np.zeros_like(g), g, cfg.nu_pre, cfg.smoother, cfg.omega, T)
        Y[level] = Section.quantize(y, B, cfg.w_y(level, Lp), on)
        if exact_s:                                       # s_{l-1} = R (A y'_l + s_l), float64
            s64[level - 1] = restrict(lv.apply(Y[level].value(np.float64), np.float64) + s64[level],
                                      np.float64)
            G[level - 1] = R[level - 1]
        elif cfg.nu_pre == 0:                             # y' = 0, s = 0: g_{l-1} = r_{l-1} (Alg. 2)
            G[level - 1] = R[level - 1]
        else:
            rc = restrict(g - lv.apply(Y[level].value(T), T), T)
            G[level - 1] = Section.quantize(rc, B, cfg.w_r(level - 1, Lp), on)
    if trace is not None:
        trace["G"] = dict(G)
        trace["Ypre"] = dict(Y)
    gc = G[lc].value(np.float64) - (s64[lc] if exact_s else 0.0)
    yc = coarse_solve(ops[lc], gc)                        # coarsest, float64
    Y[lc] = Section.quantize(yc, B, cfg.w_y(lc, Lp), on)
    U[lc] = Section.quantize(U[lc].value(np.float64) + Y[lc].value(np.float64),
                             B, cfg.w_u(lc, Lp), on)
    E = Y[lc].value(T)                                    # y'_lc + z_lc, z_lc = 0
    if trace is not None:
        trace["E"] = {}
    for level in range(lc + 1, Lp + 1):                   # coarse to fine
        lv = ops[level]
        if trace is not None:
            trace["E"][level - 1] = E
        z = prolong(E, T)
        rhs = rhs_of(level) - lv.apply(z, T)
        y = smooth(lv, Y[level].value(T), rhs, cfg.nu_post, cfg.smoother, cfg.omega, T)
        Y[level] = Section.quantize(y, B, cfg.w_y(level, Lp), on)
        U[level] = Section.quantize(U[level].value(np.float64) + Y[level].value(np.float64),
                                    B, cfg.w_u(level, Lp), on)
        if level < Lp:
            E = Y[level].value(T) + z
    return Y


def fmg_solve(f_full: np.ndarray, cfg: Config, kappa=None, history=None, levels=None):
    """Compact FMG with IR (Alg. 3).  Returns ``(u_full, U)``.

    ``f_full`` is the ``(2**L + 1)**dim`` right-hand side (boundary ignored);
    ``u_full`` the decoded FP64 solution on the same node grid (boundary 0);
    ``U`` the final compact sections.  ``history``, if a list, receives the
    float64 2-norm of each IR residual ``t`` before rounding; ``levels``, if a
    dict, receives the decoded node-grid solution after every FMG level.
    """
    lc, L = cfg.coarsest, cfg.L
    if not 1 <= lc < L:
        raise ValueError("need 1 <= coarsest < L")
    ops = hierarchy(cfg.dim, L, lc, cfg.op, kappa)
    U = {}
    yc = coarse_solve(ops[lc], inject(f_full, L, lc))
    U[lc] = Section.quantize(yc, cfg.block, cfg.w_u(lc, lc), cfg.quantize)
    for Lp in range(lc + 1, L + 1):
        for level in range(lc, Lp):
            U[level] = U[level].widen(cfg.w_u(level, Lp))
        U[Lp] = Section.zeros(cfg.dim, Lp, cfg.block, cfg.w_u(Lp, Lp), cfg.quantize)
        f_level = inject(f_full, L, Lp)
        iters = cfg.ir_iters + (cfg.final_iters if Lp == L else 0)
        for _ in range(iters):
            g = residual_hierarchy(U, f_level, ops, cfg, Lp)
            if history is not None:
                uh = decode_chain(U, lc, Lp)
                history.append(float(np.linalg.norm(f_level - ops[Lp].apply(uh, np.float64))))
            vcycle_correct(U, g, ops, cfg, Lp)
        if levels is not None:
            levels[Lp] = to_full(decode_chain(U, lc, Lp))
    return to_full(decode_chain(U, lc, L)), U


def vcycle_standard(r_full: np.ndarray, cfg: Config, kappa=None):
    """One compact V-cycle on a standard FP64 fine residual (the ``cmg_vcycle``
    entry): round ``r`` to the finest residual width (and, when the cycle
    needs them, restrict it unrounded to every level first, Alg. 2), run the
    cycle from zero on a zero solution, and return the decoded correction
    on the node grid."""
    lc, L = cfg.coarsest, cfg.L
    ops = hierarchy(cfg.dim, L, lc, cfg.op, kappa)
    r = inject(r_full, L, L)
    if chain_needed(cfg):
        g = restrict_chain(r, cfg, L, L)
    else:
        g = Section.quantize(r, cfg.block, cfg.w_r(L, L), cfg.quantize)
    U = {level: Section.zeros(cfg.dim, level, cfg.block, cfg.w_u(level, L), cfg.quantize)
         for level in range(lc, L + 1)}
    vcycle_correct(U, g, ops, cfg, L)
    return to_full(decode_chain(U, lc, L))


def storage_bits(cfg: Config) -> dict:
    """Stored bits of the sections ``u'``, ``g`` and ``y'`` on the finest FMG
    level (mantissas at their logical widths, plus 16-bit block exponents),
    the quantity of Sec. 6.1.1 and 6.1.3."""
    out = {"u": 0, "r": 0, "y": 0, "exp": 0}
    L, lc, B = cfg.L, cfg.coarsest, cfg.block
    for level in range(lc, L + 1):
        n = (1 << level) ** cfg.dim
        out["u"] += n * cfg.w_u(level, L)
        out["r"] += n * cfg.w_r(level, L)
        out["y"] += n * cfg.w_y(level, L)
        out["exp"] += 3 * 16 * bfp.n_blocks(n, B)
    return out
