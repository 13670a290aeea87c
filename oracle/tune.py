"""Precision and iteration tuning of the compact FMG — oracle (test infrastructure only).

Follows the experimental optimisation of Sec. 7.1 (Setup): with the other
constants generous (30 bits, N = 12 IR iterations), raise b2 from 1 until the
acceptance criteria hold on a small problem, add one bit and check again;
then, b2 fixed, tune b1 and finally N (from 1) the same way.  Table 1 names
four constants; b3 and b4 (matrices, f and z) are here the IEEE types of the
arithmetic (FP64 residual, FP32 V-cycle), so the search covers b2 (residual
and correction widths: bits_r = bits_y), b1 (solution width: bits_u) and N.

Acceptance (eqs. experiment-successful and experiment-successful-order, in
the finite-difference norm ``||e||_h``): for every ``L`` in ``[Lmin, Lmax]``
the compact FMG solution is within twice the discretisation error of the
closed-form discrete solution for the sine right-hand side, and for
``L >= max(Lmin + 1, 4)`` the convergence order is at least 1.95.
"""
from __future__ import annotations

import numpy as np

from oracle import compact
from oracle import grid

MAX_RY = 24    # residual / correction widths with the FP32 V-cycle
MAX_U = 53


def _sine(dim: int, L: int):
    n = 1 << L
    x = np.arange(n + 1, dtype=np.float64) / n
    s = np.sin(np.pi * x)
    s[0] = s[-1] = 0.0
    u = s
    for _ in range(dim - 1):
        u = np.multiply.outer(u, s)
    return u, dim * np.pi ** 2 * u


def errors(dim: int, Lmax: int, b1: int, b2: int, N: int, **cfg) -> dict:
    """``{L: (||u_tilde - u*||_h, ||u_h - u*||_h)}`` for ``L = 1 .. Lmax`` from
    one compact FMG run to ``Lmax`` (the state after FMG level ``L`` equals a
    run with ``Lmax = L``: the widths depend on the current FMG level only and
    the coarser right-hand sides are samples at coincident nodes)."""
    u_star, f = _sine(dim, Lmax)
    c = compact.Config(dim=dim, L=Lmax, bits_u=b1, bits_r=b2, bits_y=b2, ir_iters=N, **cfg)
    sols = {}
    compact.fmg_solve(f, c, levels=sols)
    out = {}
    for L, u in sols.items():
        h = 2.0 ** -L
        us = u_star[(slice(None, None, 1 << (Lmax - L)),) * dim]
        uh = ((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2 * us
        out[L] = (grid.norm_h(u - us, h), grid.norm_h(uh - us, h))
    return out


def accepted(dim: int, Lmin: int, Lmax: int, b1: int, b2: int, N: int, **cfg) -> bool:
    e = errors(dim, Lmax, b1, b2, N, **cfg)
    for L in range(Lmin, Lmax + 1):
        if not e[L][0] <= 2.0 * e[L][1]:
            return False
    for L in range(max(Lmin + 1, 4), Lmax + 1):
        if not -np.log2(e[L][0] / e[L - 1][0]) >= 1.95:
            return False
    return True


def _smallest(ok, lo: int, hi: int):
    """Smallest v in [lo, hi] with ok(v) such that ok(v + 1) holds too
    (the extra bit or iteration of Sec. 7.1); returns v + 1, or None."""
    v = lo
    while v < hi:
        if ok(v) and ok(v + 1):
            return v + 1
        v += 1
    return None


def tune(dim: int, Lmax: int, Lmin: int = 3, start_bits: int = 30, start_N: int = 12, **cfg) -> dict:
    """``{"bits_u": b1, "bits_r": b2, "bits_y": b2, "ir_iters": N}`` or raises."""
    b2 = _smallest(lambda b: accepted(dim, Lmin, Lmax, start_bits, b, start_N, **cfg), 2, MAX_RY)
    if b2 is None:
        raise RuntimeError("no residual width passes")
    b1 = _smallest(lambda b: accepted(dim, Lmin, Lmax, b, b2, start_N, **cfg), 2, MAX_U)
    if b1 is None:
        raise RuntimeError("no solution width passes")
    N = _smallest(lambda k: accepted(dim, Lmin, Lmax, b1, b2, k, **cfg), 1, start_N)
    if N is None:
        raise RuntimeError("no iteration count passes")
    return {"bits_u": b1, "bits_r": b2, "bits_y": b2, "ir_iters": N}
