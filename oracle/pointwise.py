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
