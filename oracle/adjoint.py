"""Adjoint solve and coefficient gradient — oracle (test infrastructure only).

Not part of the paper's method: the differentiable wrapper around it.  For
``-div(kappa grad u) = f`` with the edge discretisation of
:mod:`oracle.grid` and the loss ``J = 1/2 sum_interior (u - u_obs)**2``:

* adjoint: ``A lambda = dJ/du = u - u_obs`` (``A`` is symmetric);
* ``dJ/dkappa_e = -h**-2 (lambda_p - lambda_q)(u_p - u_q)`` for edge
  ``e = (p, q)`` (boundary values are 0);
* ``dJ/dkappa_c = 2**-(d-1) sum_{edges e of cell c} dJ/dkappa_e`` because each
  edge coefficient is the mean of the ``2**(d-1)`` cells sharing it;
* ``dJ/df = lambda``.

Summation order of the cell gradient: edges along x, then y, then z; within
one direction the ``2**(d-1)`` parallel edges of the cell in C order of
their corner offsets; each term is
``(lambda_hi - lambda_lo) * (u_hi - u_lo)``; the sum is finally multiplied
by ``-h**-2 * 2**-(d-1)``.
"""
from __future__ import annotations

import itertools

import numpy as np


def loss(u_full: np.ndarray, u_obs: np.ndarray) -> float:
    d = u_full.ndim
    inner = (slice(1, -1),) * d
    diff = u_full[inner] - u_obs[inner]
    return 0.5 * float(np.sum(diff * diff))


def loss_grad_u(u_full, u_obs):
    d = u_full.ndim
    g = np.zeros_like(u_full)
    inner = (slice(1, -1),) * d
    g[inner] = u_full[inner] - u_obs[inner]
    return g


def grad_kappa(u_full: np.ndarray, lam_full: np.ndarray) -> np.ndarray:
    """``dJ/dkappa`` on the ``(2**L)**d`` cells from node arrays ``u``, ``lambda``."""
    d = u_full.ndim
    N = u_full.shape[0]
    n = N - 1
    s = None
    for ax in reversed(range(d)):                  # x, then y, then z
        others = [a for a in range(d) if a != ax]
        for offs in itertools.product((0, 1), repeat=d - 1):
            lo = [None] * d
            hi = [None] * d
            lo[ax] = slice(0, n)
            hi[ax] = slice(1, n + 1)
            for a, o in zip(others, offs):
                lo[a] = slice(o, o + n)
                hi[a] = slice(o, o + n)
            lo, hi = tuple(lo), tuple(hi)
            t = (lam_full[hi] - lam_full[lo]) * (u_full[hi] - u_full[lo])
            s = t if s is None else s + t
    return s * (-(float(n * n)) * 0.5 ** (d - 1))
