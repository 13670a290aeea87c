"""Node-by-node evaluation of the compact residual — oracle (test infrastructure only).

At full size (1025^3) the whole-array oracle does not fit the time budget
of a test, but the IR residual (Alg. 2) at one BFP block only needs the
decode chain (eq. compact-to-standard) at the block's 64 nodes and their
stencil neighbours, and the chain at a node only needs its coarse
neighbours on the next coarser level, and so on.  This module evaluates
exactly that, with the same operations in the same order as
:mod:`oracle.compact` and :mod:`oracle.grid` (float64; prolongation terms in
C order of the coarse nodes; the stencil as centre, -x, +x, -y, +y, -z, +z),
so its values equal the whole-array oracle's bit for bit.

Nodes are given as integer arrays of padded coordinates ``(z, y, x)`` on a
level with ``n = 2**level`` intervals; coordinate ``n`` is the implicit far
boundary node (value 0).
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle import bfp


class Codes:
    """A section's raw storage: codes in their container (int8/16/32/64
    array, one entry per value; the 12-bit container is not supported
    here), int16 block exponents, block length and width."""

    def __init__(self, codes: np.ndarray, exps: np.ndarray, block: int, w: int):
        if bfp.container_bits(w) == 12:
            raise ValueError("the 12-bit container is not supported node by node")
        self.codes, self.exps, self.block, self.w = codes, np.asarray(exps, dtype=np.int64), block, w

    def at(self, flat: np.ndarray) -> np.ndarray:
        m = self.codes[flat].astype(np.int64)
        e = self.exps[flat // self.block]
        q = np.where(e == bfp.ZERO_EXP, 0, e - (self.w - 1))
        return np.where(e == bfp.ZERO_EXP, 0.0, np.ldexp(m.astype(np.float64), q))


def _flat(idx: np.ndarray, n: int) -> np.ndarray:
    z, y, x = idx[:, 0].astype(np.int64), idx[:, 1].astype(np.int64), idx[:, 2].astype(np.int64)
    return (z * n + y) * n + x


def decode_chain_at(U: dict, lc: int, level: int, idx: np.ndarray) -> np.ndarray:
    """``u_level`` (float64) at the nodes ``idx`` (shape ``(k, 3)``)."""
    n = 1 << level
    idx = np.asarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0])
    inside = ~np.any(idx == n, axis=1)       # far-boundary nodes stay 0
    node = idx[inside]
    val = U[level].at(_flat(node, n))
    if level == lc:
        out[inside] = val
        return out
    par, base = node & 1, node >> 1
    w = np.prod(np.where(par == 1, 0.5, 1.0), axis=1)  # every term of a node has this weight
    # coarse neighbours of every node, in C order of the (z, y, x) offsets
    terms = []
    for o in itertools.product((0, 1), repeat=3):
        o = np.array(o)
        terms.append((np.all((o == 0) | (par == 1), axis=1), base + o))
    need = np.unique(np.concatenate([c[u] for u, c in terms]), axis=0)
    coarse = decode_chain_at(U, lc, level - 1, need)
    m1 = (n >> 1) + 1
    key = _flat(need, m1)
    order = np.argsort(key)
    key, coarse = key[order], coarse[order]
    s = None
    for use, c in terms:
        pos = np.searchsorted(key, _flat(np.where(use[:, None], c, base), m1))
        t = w * coarse[pos]
        s = t if s is None else np.where(use, s + t, s)
    out[inside] = val + s
    return out


def ir_residual_block(U: dict, lc: int, L: int, f_block: np.ndarray, z: int, y: int, bx: int, block: int,
                      w: int):
    """Codes and exponent of the residual section ``g_L = Q_w(f - A u_L)``
    (Alg. 2) at the block of ``block`` nodes starting at ``x = bx * block``
    of row ``(z, y)``; ``f_block`` holds f at those nodes (boundary entries
    ignored)."""
    n = 1 << L
    x = bx * block + np.arange(block)
    centre = np.stack([np.full(block, z), np.full(block, y), x], axis=1)
    offsets = [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]
    nodes = [centre] + [centre + np.array(o) for o in offsets]
    allv = decode_chain_at(U, lc, L, np.clip(np.concatenate(nodes), 0, n))
    u = allv.reshape(7, block)
    s = 6.0 * u[0]
    for k in range(1, 7):
        s = s - u[k]
    au = s * float(4 ** L)
    interior = (x >= 1) & (z >= 1) & (y >= 1)
    t = np.where(interior, np.asarray(f_block, dtype=np.float64) - au, 0.0)
    m, e = bfp.encode(t, block, w)
    return m, int(e[0])


# --------------------------------------------------- the down sweep, locally
def _apply_box(y: np.ndarray, level: int, T) -> np.ndarray:
    """Poisson ``A y`` at the inner nodes of a box (all six neighbours in the
    box), the terms in the order of :meth:`oracle.grid.Level.apply`; 0 on the
    box's outer shell."""
    out = np.zeros_like(y)
    c = (slice(1, -1),) * 3
    s = T(6) * y[c]
    for ax in (2, 1, 0):                     # -x, +x, -y, +y, -z, +z
        for off in (-1, 1):
            sl = [slice(1, -1)] * 3
            sl[ax] = slice(1 + off, y.shape[ax] - 1 + off)
            s = s - y[tuple(sl)]
    out[c] = s * T(4 ** level)
    return out


def rbgs_box(g: np.ndarray, origin, level: int, nu: int, T=np.float32) -> np.ndarray:
    """``nu`` red-black Gauss-Seidel sweeps from ``y = 0`` on ``A y = g``
    restricted to a box of level ``level`` whose node ``[0, 0, 0]`` has the
    padded coordinates ``origin`` (the box may hold far-boundary nodes ``n``).
    Same arithmetic as :func:`oracle.grid.smooth` (red = even parity first,
    ``c = 1 / (6 * 4**level)`` rounded to ``T``).  Nodes on the box's outer
    shell keep 0, so values are exact at depth greater than ``2 nu`` inside
    the box (each half-sweep carries information one node)."""
    n = 1 << level
    rhs = np.asarray(g, dtype=T)
    y = np.zeros_like(rhs)
    cz, cy, cx = (origin[a] + np.arange(rhs.shape[a]) for a in range(3))
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    interior = (Z >= 1) & (Z < n) & (Y >= 1) & (Y < n) & (X >= 1) & (X < n)
    inner = np.zeros(rhs.shape, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    c = T(1.0 / (2 * 3 * float(4 ** level)))
    for _ in range(nu):
        for colour in (0, 1):
            mask = interior & inner & (((Z + Y + X) % 2) == colour)
            r = rhs - _apply_box(y, level, T)
            y[mask] = y[mask] + c * r[mask]
    return y


def down_sweep_block(G: Codes, level: int, nu: int, z: int, y: int, bx: int, block: int, w: int,
                     T=np.float32):
    """Codes and exponent of ``y'_level = Q_w(S^nu(0; g))`` (generalised
    Alg. 1, fine to coarse) at one block, from the residual section ``G``."""
    n = 1 << level
    M = 2 * nu + 1
    x0 = bx * block
    lo = np.array([z - M, y - M, x0 - M])
    hi = np.array([z + M, y + M, x0 + block - 1 + M])
    lo_c, hi_c = np.maximum(lo, 0), np.minimum(hi, n)
    gb = _box_values(G, level, lo_c, hi_c, T)
    yb = rbgs_box(gb, lo_c, level, nu, T)
    row = yb[z - lo_c[0], y - lo_c[1], x0 - lo_c[2]: x0 - lo_c[2] + block]
    m, e = bfp.encode(row.astype(np.float64), block, w)
    return m, int(e[0])


def _box_values(S: Codes, level: int, lo, hi, T) -> np.ndarray:
    """Decoded values (in ``T``) of a section on the box ``lo .. hi``
    (inclusive padded coordinates; far-boundary nodes are 0)."""
    n = 1 << level
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    Zc, Yc, Xc = np.meshgrid(*axes, indexing="ij")
    idx = np.stack([Zc.ravel(), Yc.ravel(), Xc.ravel()], axis=1)
    far = np.any(idx == n, axis=1)
    v = np.zeros(idx.shape[0])
    v[~far] = S.at(_flat(idx[~far], n))
    return v.reshape(Zc.shape).astype(T)


def restrict_block(G: Codes, level: int, nu: int, Kc: int, Jc: int, bxc: int, block: int, w_y: int, w_r: int,
                   T=np.float32):
    """Codes and exponent of ``g_{level-1} = Q_{w_r}(R(g - A y'))`` at one
    block of the coarse level (coarse row ``(Kc, Jc)``, x from
    ``bxc * block``), with ``y' = Q_{w_y}(S^nu(0; g))`` formed locally: the
    fine-to-coarse step of the generalised Alg. 1 written for ``g = r - s``."""
    n, m = 1 << level, 1 << (level - 1)
    M = 2 * nu + 1
    fx0 = 2 * bxc * block
    # fine rows whose y' enters: 2Kc-2 .. 2Kc+2, 2Jc-2 .. 2Jc+2; x over the
    # fine blocks covering 2 bxc*block - 2 .. 2 (bxc+1)*block
    xb0 = max(0, (fx0 - 2) // block)
    xb1 = min(n // block - 1, (fx0 + 2 * block) // block)
    lo = np.array([2 * Kc - 2 - M, 2 * Jc - 2 - M, xb0 * block - M])
    hi = np.array([2 * Kc + 2 + M, 2 * Jc + 2 + M, (xb1 + 1) * block - 1 + M])
    lo_c, hi_c = np.maximum(lo, 0), np.minimum(hi, n)
    gb = _box_values(G, level, lo_c, hi_c, T)
    yb = rbgs_box(gb, lo_c, level, nu, T)
    # y' on whole fine blocks of the rows 2Kc-2 .. 2Kc+2, 2Jc-2 .. 2Jc+2
    yq = np.zeros_like(yb)
    for fz in range(max(0, 2 * Kc - 2), min(n - 1, 2 * Kc + 2) + 1):
        for fy in range(max(0, 2 * Jc - 2), min(n - 1, 2 * Jc + 2) + 1):
            for xb in range(xb0, xb1 + 1):
                a = xb * block - lo_c[2]
                row = yb[fz - lo_c[0], fy - lo_c[1], a: a + block].astype(np.float64)
                mq, eq = bfp.encode(row, block, w_y)
                yq[fz - lo_c[0], fy - lo_c[1], a: a + block] = bfp.decode(mq, eq, block, w_y, dtype=T)
    # t = g - A y' at the fine nodes 2K-1 .. 2K+1 (boundary nodes: t = g = 0)
    t = gb - _apply_box(yq, level, T)
    cz, cy, cx = (lo_c[a] + np.arange(gb.shape[a]) for a in range(3))
    Zf, Yf, Xf = np.meshgrid(cz, cy, cx, indexing="ij")
    t = np.where((Zf >= 1) & (Zf < n) & (Yf >= 1) & (Yf < n) & (Xf >= 1) & (Xf < n), t, gb)
    # full weighting of the coarse row, terms in C order of the offsets
    I = bxc * block + np.arange(block)
    s = None
    for oz, oy, ox in itertools.product((-1, 0, 1), repeat=3):
        wgt = (0.5 if oz == 0 else 0.25) * (0.5 if oy == 0 else 0.25) * (0.5 if ox == 0 else 0.25)
        fz, fy, fx = 2 * Kc + oz, 2 * Jc + oy, 2 * I + ox
        v = t[fz - lo_c[0], fy - lo_c[1], np.clip(fx - lo_c[2], 0, t.shape[2] - 1)]
        term = T(wgt) * v
        s = term if s is None else s + term
    inside = (I >= 1) & (I < m) & (Kc >= 1) & (Kc < m) & (Jc >= 1) & (Jc < m)
    c = np.where(inside, s, T(0)).astype(np.float64)
    mq, eq = bfp.encode(c, block, w_r)
    return mq, int(eq[0])


# ----------------------------------------------------- the up sweep, locally
def prolong_box(E: np.ndarray, lo, hi, T=np.float32) -> np.ndarray:
    """``z = P E`` (d-linear interpolation of the coarse array ``E``, padded
    layout of the next coarser level) on the fine box ``lo .. hi`` (inclusive
    padded coordinates; the far-boundary node ``n`` is 0).  Terms as in
    :func:`oracle.grid.prolong`: weight ``T(w)`` times the coarse value, the
    coarse neighbours in C order of their (z, y, x) offsets."""
    m = E.shape[0]
    n = 2 * m
    ce = np.pad(np.asarray(E, dtype=T), [(0, 1)] * 3)
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    idx = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    out = np.zeros(idx.shape[:3], dtype=T)
    par, base = idx & 1, idx >> 1
    for pz, py, px in itertools.product((0, 1), repeat=3):
        sel = (par[..., 0] == pz) & (par[..., 1] == py) & (par[..., 2] == px) & np.all(idx < n, axis=-1)
        if not sel.any():
            continue
        b = base[sel]
        per_axis = [[(0, 1.0)] if p == 0 else [(0, 0.5), (1, 0.5)] for p in (pz, py, px)]
        s = None
        for combo in itertools.product(*per_axis):
            w = combo[0][1] * combo[1][1] * combo[2][1]
            t = T(w) * ce[b[:, 0] + combo[0][0], b[:, 1] + combo[1][0], b[:, 2] + combo[2][0]]
            s = t if s is None else s + t
        out[sel] = s
    return out


def up_sweep_block(G: Codes, Y: Codes, U: Codes, E: np.ndarray, level: int, nu: int, z: int, y: int, bx: int,
                   block: int, w_y: int, w_u: int, T=np.float32):
    """The up sweep and correction of level ``level`` (Alg. 1 coarse to
    fine; Alg. 3 apply correction) at one block: ``z = P E``,
    ``y = S^nu(dec y'_pre; dec g - A z)`` (red-black Gauss-Seidel in ``T``),
    ``y' = Q_{w_y}(y)`` and ``u' = Q_{w_u}(dec u' + dec y')`` in float64.
    Red-black sweeps carry information one node per half-sweep, so a box of
    radius ``2 nu + 1`` around the block (its outer shell held fixed) gives
    the whole-array values at the block.  Returns
    ``(y' codes, y' exponent, u' codes, u' exponent)``."""
    n = 1 << level
    M = 2 * nu + 1
    x0 = bx * block
    lo = np.array([z - M, y - M, x0 - M])
    hi = np.array([z + M, y + M, x0 + block - 1 + M])
    lo_c, hi_c = np.maximum(lo, 0), np.minimum(hi, n)
    zb = prolong_box(E, lo_c, hi_c, T)
    rhs = _box_values(G, level, lo_c, hi_c, T) - _apply_box(zb, level, T)
    yb = _box_values(Y, level, lo_c, hi_c, T)
    cz, cy, cx = (lo_c[a] + np.arange(yb.shape[a]) for a in range(3))
    Zc, Yc, Xc = np.meshgrid(cz, cy, cx, indexing="ij")
    interior = (Zc >= 1) & (Zc < n) & (Yc >= 1) & (Yc < n) & (Xc >= 1) & (Xc < n)
    inner = np.zeros(yb.shape, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    c = T(1.0 / (2 * 3 * float(4 ** level)))
    for _ in range(nu):
        for colour in (0, 1):
            mask = interior & inner & (((Zc + Yc + Xc) % 2) == colour)
            r = rhs - _apply_box(yb, level, T)
            yb[mask] = yb[mask] + c * r[mask]
    row = yb[z - lo_c[0], y - lo_c[1], x0 - lo_c[2]: x0 - lo_c[2] + block].astype(np.float64)
    my, ey = bfp.encode(row, block, w_y)
    dy = bfp.decode(my, ey, block, w_y, dtype=np.float64)
    flat = (z * n + y) * n + x0 + np.arange(block)
    mu, eu = bfp.encode(U.at(flat) + dy, block, w_u)
    return my, int(ey[0]), mu, int(eu[0])
