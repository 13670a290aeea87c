"""Tuning of the precision constants and the IR iteration count.

The experimental optimisation of Sec. 7.1 (Setup), run with the library's
solver on a small problem: with the other constants generous (30 bits,
N = 12), raise the residual/correction width b2 from 2 until the acceptance
criteria hold, add one bit (and require the criteria still hold); then, b2
fixed, tune the solution width b1 and finally the iteration count N (from 1)
the same way.  The matrix and right-hand-side precisions b3, b4 of Table 1
are the IEEE types of the arithmetic here, so they are not searched.

Acceptance (Sec. 7.1, in the finite-difference norm ``||e||_h``) on the
manufactured problem ``-Laplace u = d pi^2 prod sin(pi x_i)`` with zero
Dirichlet data: for every ``L`` in ``[Lmin, Lmax]`` the FMG solution lies
within twice the discretisation error of the exact discrete solution
``((pi h / 2) / sin(pi h / 2))^2 u*``, and for ``L >= max(Lmin + 1, 4)`` the
error decreases at order >= 1.95.
"""
from __future__ import annotations

import math

MAX_RY = 24   # residual / correction widths with the FP32 V-cycle
MAX_U = 53


def _sine_problem(dim: int, L: int):
    import torch
    n = 1 << L
    x = torch.arange(n + 1, dtype=torch.float64, device="cuda") / n
    s = torch.sin(math.pi * x)
    s[0] = 0.0
    s[-1] = 0.0
    u = s
    for _ in range(dim - 1):
        u = u[..., None] * s
    return u, (dim * math.pi ** 2) * u


def errors(dim: int, L: int, b1: int, b2: int, N: int, **opts):
    """``(||u_tilde - u*||_h, ||u_h - u*||_h)`` of one compact FMG solve."""
    import torch

    from . import Solver
    h = 2.0 ** -L
    us, f = _sine_problem(dim, L)
    with Solver(dim, L, bits_u=b1, bits_r=b2, bits_y=b2, ir_iters=N, **opts) as s:
        u = s.solve(f[None].contiguous())[0]
    ch = ((math.pi * h / 2) / math.sin(math.pi * h / 2)) ** 2
    norm = lambda e: math.sqrt(h ** dim * float(torch.sum(e * e)))  # noqa: E731
    return norm(u - us), norm((ch - 1.0) * us)


def accepted(dim: int, Lmin: int, Lmax: int, b1: int, b2: int, N: int, **opts) -> bool:
    e = {L: errors(dim, L, b1, b2, N, **opts) for L in range(Lmin, Lmax + 1)}
    if any(not e[L][0] <= 2.0 * e[L][1] for L in e):
        return False
    return all(-math.log2(e[L][0] / e[L - 1][0]) >= 1.95 for L in range(max(Lmin + 1, 4), Lmax + 1))


def _with_margin(ok, lo: int, hi: int):
    """The smallest passing value plus one, where that value passes too."""
    for v in range(lo, hi):
        if ok(v) and ok(v + 1):
            return v + 1
    return None


def tune_widths(dim: int = 3, Lmax: int = 5, Lmin: int = 3, start_bits: int = 30, start_N: int = 12,
                **opts) -> dict:
    """Return ``{"bits_u", "bits_r", "bits_y", "ir_iters"}`` for a problem
    class; ``opts`` are further solver options (smoother, omega, bfp_block,
    nu_pre, nu_post).  Raises ``RuntimeError`` if no setting passes."""
    b2 = _with_margin(lambda b: accepted(dim, Lmin, Lmax, start_bits, b, start_N, **opts), 2, MAX_RY)
    if b2 is None:
        raise RuntimeError("no residual width passes the acceptance test")
    b1 = _with_margin(lambda b: accepted(dim, Lmin, Lmax, b, b2, start_N, **opts), 2, MAX_U)
    if b1 is None:
        raise RuntimeError("no solution width passes the acceptance test")
    N = _with_margin(lambda k: accepted(dim, Lmin, Lmax, b1, b2, k, **opts), 1, start_N)
    if N is None:
        raise RuntimeError("no iteration count passes the acceptance test")
    return {"bits_u": b1, "bits_r": b2, "bits_y": b2, "ir_iters": N}
