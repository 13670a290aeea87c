"""Dense matrices on tiny grids — oracle (test infrastructure only).

Written from the textbook definitions, independently of :mod:`oracle.grid`,
so that the vectorised operators can be checked against them: Kronecker
sums of the 1-D second difference, Kronecker products of 1-D linear
interpolation, and an edge-by-edge assembly of the diffusion matrix.
Unknowns are the interior nodes in C order (x fastest).
"""
from __future__ import annotations

import itertools

import numpy as np


def second_difference_1d(level: int) -> np.ndarray:
    n = 1 << level
    m = n - 1
    T = 2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    return T * float(n * n)


def poisson(dim: int, level: int) -> np.ndarray:
    """``-Laplace`` on the interior nodes: a Kronecker sum of 1-D operators."""
    T = second_difference_1d(level)
    I = np.eye(T.shape[0])
    if dim == 2:
        return np.kron(I, T) + np.kron(T, I)
    return np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)


def interpolation_1d(level: int) -> np.ndarray:
    """Linear interpolation from level ``level-1`` to ``level`` (interiors)."""
    n = 1 << level
    m = n // 2
    P = np.zeros((n - 1, m - 1))
    for j in range(1, m):              # coarse interior node j at fine 2j
        P[2 * j - 1, j - 1] = 1.0
        P[2 * j - 2, j - 1] += 0.5
        P[2 * j, j - 1] += 0.5
    return P


def prolongation(dim: int, level: int) -> np.ndarray:
    P = interpolation_1d(level)
    out = P
    for _ in range(dim - 1):
        out = np.kron(out, P)
    return out


def diffusion(kappa: np.ndarray) -> np.ndarray:
    """Assemble ``-div(kappa grad)`` edge by edge.

    Every grid edge ``e = (p, q)`` carries ``k_e`` = mean of the cells that
    share it and contributes ``k_e h**-2 (u_p - u_q)`` to row ``p`` and the
    negative to row ``q``; rows and columns of boundary nodes are dropped.
    """
    d = kappa.ndim
    n = kappa.shape[0]
    h2 = float(n * n)
    m = n - 1
    idx = {}
    for k, node in enumerate(itertools.product(range(1, n), repeat=d)):
        idx[node] = k
    A = np.zeros((m ** d, m ** d))
    for node in itertools.product(range(0, n + 1), repeat=d):
        for ax in range(d):
            q = list(node)
            q[ax] += 1
            if q[ax] > n:
                continue
            q = tuple(q)
            # cells sharing the edge: index node[ax] on ax, node[a]-1 or node[a] elsewhere
            cells = []
            others = [a for a in range(d) if a != ax]
            for offs in itertools.product((-1, 0), repeat=d - 1):
                c = list(node)
                ok = True
                for a, o in zip(others, offs):
                    c[a] = node[a] + o
                    if not 0 <= c[a] < n:
                        ok = False
                if ok:
                    cells.append(kappa[tuple(c)])
            if len(cells) != 2 ** (d - 1):
                continue                      # edge on the boundary surface
            ke = float(np.mean(cells)) * h2
            ip, iq = idx.get(node), idx.get(q)
            if ip is not None:
                A[ip, ip] += ke
            if iq is not None:
                A[iq, iq] += ke
            if ip is not None and iq is not None:
                A[ip, iq] -= ke
                A[iq, ip] -= ke
    return A


def diffusion_derivative(kappa: np.ndarray, cell) -> np.ndarray:
    """``dA/dkappa_c`` for one cell, by differencing the linear map exactly:
    ``A`` is linear in ``kappa``, so ``A(e_c)`` is the derivative."""
    e = np.zeros_like(kappa)
    e[cell] = 1.0
    return diffusion(e)


def interior(u: np.ndarray) -> np.ndarray:
    d = u.ndim
    return u[(slice(1, -1),) * d].reshape(-1)
