"""Level grids, operators, transfers and smoothers — oracle (test infrastructure only).

The multigrid components the paper assumes (Sec. 3.1): a system matrix per
level, prolongation ``P_l`` from level ``l-1`` to ``l``, restriction ``R_l``
and a smoother of the form ``y <- y + M (r - A y)`` (eq. smoother).  The
paper discretises with B-spline finite elements and Galerkin coarse
operators; the workloads here use finite differences rediscretised on every
level, d-linear interpolation and full weighting ``R = 2**-d P^T``.

Level layout (the "padded" layout): level ``l`` has ``n = 2**l`` intervals
per axis and is stored as an array of shape ``(n,)*dim`` indexed
``[z, y, x]`` (x fastest).  Index 0 on each axis is the Dirichlet boundary
node and always holds 0; the far boundary node ``n`` is implicit (0).
Interior nodes are ``1 .. n-1`` on every axis.  ``h = 2**-l``.

Floating-point conventions (so that another implementation can reproduce
the rounding exactly); ``T`` is the arithmetic type (float32 or float64):

* a stencil sums its neighbour terms in the order -x, +x, -y, +y, -z, +z;
* Poisson: ``(A u)_p = (2d*u_p - u_-x - u_+x - ...) * 4**l``;
* diffusion: ``(A u)_p = (sum_dir k_dir * (u_p - u_q)) * 4**l`` with the edge
  coefficient ``k_dir`` the mean of the ``2**(d-1)`` cells sharing the edge
  (summed in C order of the cells, then times ``2**-(d-1)``);
* prolongation: a fine node is the sum of its weighted coarse neighbours in
  C order of the coarse nodes (weights 1, 1/2, 1/4, 1/8, exact);
* restriction: full weighting, terms in C order of the offsets -1, 0, +1;
* smoothing: ``y + c * (rhs - A y)``; Poisson ``c = omega / (2d * 4**l)``
  formed in float64 and rounded to ``T``; diffusion ``c_p = omega / diag_p``
  in ``T``.  Red-black Gauss-Seidel updates the even-parity ("red") nodes
  first, then the odd ones, with ``omega = 1``.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def inv_h2(level: int) -> float:
    return float(4 ** level)


def _ext(u: np.ndarray) -> np.ndarray:
    """Append the implicit far-boundary node (value 0) on every axis."""
    return np.pad(u, [(0, 1)] * u.ndim)


def _inner(d: int, n: int, ax: int = 0, off: int = 0):
    """Slices selecting interior nodes ``1..n-1``, shifted by ``off`` on ``ax``."""
    s = [slice(1, n)] * d
    s[ax] = slice(1 + off, n + off)
    return tuple(s)


def _dirs(d: int):
    """Stencil directions in the fixed order -x, +x, -y, +y, -z, +z."""
    for ax in reversed(range(d)):
        yield ax, 0, -1
        yield ax, 1, +1


# ---------------------------------------------------------------- operators
class Level:
    """The finite-difference operator of one level (Poisson or diffusion).

    For diffusion ``kappa`` is the float64 cell array of this level.
    """

    def __init__(self, dim: int, level: int, op: str = "poisson", kappa=None):
        self.dim, self.level, self.op = dim, level, op
        self.n = 1 << level
        if op == "diffusion":
            if kappa is None or kappa.shape != (self.n,) * dim:
                raise ValueError("diffusion needs the cell coefficients of the level")
            self.kappa = np.asarray(kappa, dtype=np.float64)
        elif op != "poisson":
            raise ValueError(op)
        self._edges = {}

    # edge coefficients k_dir at every interior node, in arithmetic type T
    def edges(self, T):
        key = np.dtype(T).name
        if key not in self._edges:
            d, n = self.dim, self.n
            k = self.kappa.astype(T)
            out = {}
            for ax, side, _ in _dirs(d):
                others = [a for a in range(d) if a != ax]
                s = None
                for offs in itertools.product((-1, 0), repeat=d - 1):
                    sl = [None] * d
                    sl[ax] = slice(side, side + n - 1)   # cell i-1 (minus) or i (plus)
                    for a, o in zip(others, offs):
                        sl[a] = slice(1 + o, n + o)
                    t = k[tuple(sl)]
                    s = t if s is None else s + t
                out[(ax, side)] = s * T(0.5 ** (d - 1))
            self._edges[key] = out
        return self._edges[key]

    def apply(self, u: np.ndarray, T) -> np.ndarray:
        """``A u`` on the interior; the boundary entries of the result are 0."""
        d, n = self.dim, self.n
        ue = _ext(np.asarray(u, dtype=T))
        c = _inner(d, n)
        if self.op == "poisson":
            s = T(2 * d) * ue[c]
            for ax, _, off in _dirs(d):
                s = s - ue[_inner(d, n, ax, off)]
        else:
            ke = self.edges(T)
            up = ue[c]
            s = None
            for ax, side, off in _dirs(d):
                t = ke[(ax, side)] * (up - ue[_inner(d, n, ax, off)])
                s = t if s is None else s + t
        out = np.zeros((n,) * d, dtype=T)
        out[c] = s * T(inv_h2(self.level))
        return out

    def diag(self, T) -> np.ndarray:
        """Diagonal of ``A`` on the interior nodes (shape ``(n-1,)*dim``)."""
        d, n = self.dim, self.n
        if self.op == "poisson":
            return np.full((n - 1,) * d, T(2 * d * inv_h2(self.level)), dtype=T)
        ke = self.edges(T)
        s = None
        for ax, side, _ in _dirs(d):
            t = ke[(ax, side)]
            s = t if s is None else s + t
        return s * T(inv_h2(self.level))

    def smoother_coeff(self, omega: float, T):
        """``c`` of ``y <- y + c (rhs - A y)``: scalar (Poisson) or per node."""
        if self.op == "poisson":
            return T(omega / (2 * self.dim * inv_h2(self.level)))
        return T(omega) / self.diag(T)


def coarsen_kappa(kappa: np.ndarray) -> np.ndarray:
    """Coarse cell coefficient = mean of its ``2**d`` children (C order, FP64)."""
    d = kappa.ndim
    s = None
    for offs in itertools.product((0, 1), repeat=d):
        t = kappa[tuple(slice(o, None, 2) for o in offs)]
        s = t if s is None else s + t
    return s * (0.5 ** d)


def hierarchy(dim: int, L: int, lc: int, op: str = "poisson", kappa=None):
    """Operators for levels ``lc .. L`` (kappa given on the finest cells)."""
    levels = {}
    k = None if kappa is None else np.asarray(kappa, dtype=np.float64)
    for level in range(L, lc - 1, -1):
        levels[level] = Level(dim, level, op, k)
        if k is not None and level > lc:
            k = coarsen_kappa(k)
    return levels


# ---------------------------------------------------------------- transfers
def prolong(coarse: np.ndarray, T) -> np.ndarray:
    """d-linear interpolation ``P`` from ``(m,)*d`` to ``(2m,)*d``."""
    d, m = coarse.ndim, coarse.shape[0]
    n = 2 * m
    ce = _ext(np.asarray(coarse, dtype=T))
    fine = np.zeros((n,) * d, dtype=T)
    for par in itertools.product((0, 1), repeat=d):
        per_axis = [[(0, 1.0)] if p == 0 else [(0, 0.5), (1, 0.5)] for p in par]
        s = None
        for combo in itertools.product(*per_axis):
            w = math.prod(wt for _, wt in combo)
            t = T(w) * ce[tuple(slice(o, o + m) for o, _ in combo)]
            s = t if s is None else s + t
        fine[tuple(slice(p, n, 2) for p in par)] = s
    return fine


def restrict(fine: np.ndarray, T) -> np.ndarray:
    """Full weighting ``R = 2**-d P^T`` from ``(2m,)*d`` to ``(m,)*d``."""
    d, n = fine.ndim, fine.shape[0]
    m = n // 2
    fl = np.asarray(fine, dtype=T)
    s = None
    for offs in itertools.product((-1, 0, 1), repeat=d):
        w = math.prod(0.5 if o == 0 else 0.25 for o in offs)
        t = T(w) * fl[tuple(slice(2 + o, 2 * m - 1 + o, 2) for o in offs)]
        s = t if s is None else s + t
    coarse = np.zeros((m,) * d, dtype=T)
    coarse[(slice(1, m),) * d] = s
    return coarse


# ---------------------------------------------------------------- smoothers
def _colour_mask(d: int, n: int, colour: int) -> np.ndarray:
    idx = np.indices((n,) * d).sum(axis=0)
    mask = (idx % 2) == colour
    for ax in range(d):
        sl = [slice(None)] * d
        sl[ax] = 0
        mask[tuple(sl)] = False
    return mask


def smooth(lv: Level, y: np.ndarray, rhs: np.ndarray, nu: int, smoother: str,
           omega: float, T) -> np.ndarray:
    """``nu`` sweeps of weighted Jacobi or red-black Gauss-Seidel on ``A y = rhs``."""
    y = np.array(y, dtype=T, copy=True)
    rhs = np.asarray(rhs, dtype=T)
    d, n = lv.dim, lv.n
    inner = _inner(d, n)
    if smoother == "wjacobi":
        c = lv.smoother_coeff(omega, T)
        for _ in range(nu):
            r = rhs[inner] - lv.apply(y, T)[inner]
            y[inner] = y[inner] + c * r
        return y
    if smoother != "rbgs":
        raise ValueError(smoother)
    c = lv.smoother_coeff(1.0, T)
    c_full = None
    if not np.isscalar(c) and np.ndim(c) > 0:
        c_full = np.zeros((n,) * d, dtype=T)
        c_full[inner] = c
    for _ in range(nu):
        for colour in (0, 1):
            mask = _colour_mask(d, n, colour)
            r = rhs - lv.apply(y, T)
            cm = c if c_full is None else c_full[mask]
            y[mask] = y[mask] + cm * r[mask]
    return y


def ldlt_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve ``A x = b`` for symmetric positive definite ``A`` in float64:
    ``A = L D L^T`` with unit lower-triangular ``L`` and diagonal ``D``
    (``d_j = a_jj - sum_k l_jk^2 d_k``, ``l_ij = (a_ij - sum_k l_ik l_jk d_k)
    / d_j``), then ``L z = b``, ``L^T x = D^-1 z``; every sum is taken in
    increasing index order, one operation at a time."""
    m = len(b)
    Lf = [[0.0] * m for _ in range(m)]
    d = [0.0] * m
    for j in range(m):
        s = float(A[j][j])
        for k in range(j):
            s = s - (Lf[j][k] * Lf[j][k]) * d[k]
        d[j] = s
        for i in range(j + 1, m):
            t = float(A[i][j])
            for k in range(j):
                t = t - (Lf[i][k] * Lf[j][k]) * d[k]
            Lf[i][j] = t / d[j]
    z = [0.0] * m
    for i in range(m):
        s = float(b[i])
        for k in range(i):
            s = s - Lf[i][k] * z[k]
        z[i] = s
    x = [0.0] * m
    for i in range(m - 1, -1, -1):
        s = z[i] / d[i]
        for k in range(i + 1, m):
            s = s - Lf[k][i] * x[k]
        x[i] = s
    return np.array(x)


def coarse_solve(lv: Level, g: np.ndarray) -> np.ndarray:
    """Exact FP64 solve on the coarsest level (Alg. 3, coarse-grid solve).

    One interior node: ``g / diag``.  Otherwise the interior system is
    assembled column by column from :meth:`Level.apply` and solved by the
    ``L D L^T`` factorisation of :func:`ldlt_solve` (the matrix is symmetric
    positive definite).
    """
    d, n = lv.dim, lv.n
    inner = _inner(d, n)
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros((n,) * d)
    if n == 2:
        out[inner] = g[inner] / lv.diag(np.float64)
        return out
    m = (n - 1) ** d
    A = np.zeros((m, m))
    for j in range(m):
        e_in = np.zeros((n - 1,) * d)
        e_in.flat[j] = 1.0
        e = np.zeros((n,) * d)
        e[inner] = e_in
        A[:, j] = lv.apply(e, np.float64)[inner].reshape(-1)
    out[inner] = ldlt_solve(A, g[inner].reshape(-1)).reshape((n - 1,) * d)
    return out


def inject(f_full: np.ndarray, L: int, level: int) -> np.ndarray:
    """Right-hand side on FMG level ``level``: the finest array sampled at the
    coincident nodes, in the padded layout, boundary set to 0 (the
    finite-difference reading of ``discretize`` in Alg. 3)."""
    s = 1 << (L - level)
    n = 1 << level
    d = f_full.ndim
    f = np.array(f_full[(slice(0, None, s),) * d][(slice(0, n),) * d], dtype=np.float64)
    for ax in range(d):
        sl = [slice(None)] * d
        sl[ax] = 0
        f[tuple(sl)] = 0.0
    return f


def to_full(u: np.ndarray) -> np.ndarray:
    """Padded level array -> full ``(n+1)**d`` node array (far boundary 0)."""
    return _ext(u)


def norm_h(e: np.ndarray, h: float) -> float:
    """Discrete L2 norm ``(h**d * sum e**2)**(1/2)``."""
    return float(np.sqrt(h ** e.ndim * np.sum(np.asarray(e, dtype=np.float64) ** 2)))
