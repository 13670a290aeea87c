"""Adaptive-exponent BFP codec — oracle (test infrastructure only).

Sec. 6.1.3 ("Exponents") avoids knowing the block exponent in advance: the
entries of a vector are visited in order, each is normalised to the largest
exponent seen so far, and a new block (with a new exponent) starts whenever
a larger exponent turns up.  Only the ``b`` largest exponents need to be
kept, ``b`` the mantissa width: every other block's exponent is at least
``b`` below the largest, so its entries would round to zero in
single-exponent (scaled fixed-point) BFP anyway.

Readings fixed here (the paper describes the scheme in words only):

* the exponent of an entry is the fixed-block exponent of a block holding
  that entry alone: the ``frexp`` exponent of ``|x|``, plus one if ``|x|``
  rounds to ``2**(w-1)`` at width ``w``; zero has no exponent;
* the running exponent ``R_i`` is the largest entry exponent over
  ``x_0 .. x_i``; a block starts at every ``i`` where ``R_i`` rises (the
  first nonzero entry starts the first block);
* code ``m_i = RNE(x_i * 2**((w - 1) - R_i))``, 0 while no entry was
  nonzero; ``w`` counts the sign bit, codes lie in
  ``[-(2**(w-1) - 1), 2**(w-1) - 1]``;
* the kept blocks are the last ``min(#blocks, w)`` ones (their exponents
  are the ``w`` largest, since the exponents rise with the start index);
  entries before the first kept block decode to zero, whatever their
  stored code;
* codes use the containers of :mod:`oracle.bfp`; a block is an int64 start
  index and an int16 exponent.
"""
from __future__ import annotations

import numpy as np

from oracle import bfp

NO_EXP = np.iinfo(np.int64).min  # "no exponent yet": below every real one


def entry_exponents(x: np.ndarray, w: int) -> np.ndarray:
    """Exponent of each entry at width ``w`` (``NO_EXP`` for zero)."""
    bfp.container_bits(w)
    a = np.abs(np.asarray(x, dtype=np.float64).reshape(-1))
    _, e = np.frexp(a)
    e = e.astype(np.int64)
    top = np.rint(np.ldexp(a, (w - 1) - e))
    e = np.where(top == float(1 << (w - 1)), e + 1, e)
    return np.where(a == 0.0, NO_EXP, e)


def encode(x: np.ndarray, w: int):
    """``(m, starts, exps)``: int64 codes of every entry, and the kept blocks
    (int64 start indices, int16 exponents) in increasing order."""
    x = np.asarray(x).reshape(-1)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite value in BFP input")
    xd = x.astype(np.float64)
    e = entry_exponents(xd, w)
    R = np.maximum.accumulate(e) if e.size else e     # the running exponent
    prev = np.concatenate(([NO_EXP], R[:-1])) if R.size else R
    first = np.nonzero(R > prev)[0]                    # where a block starts
    seen = R != NO_EXP
    q = np.where(seen, (w - 1) - R, 0)
    m = np.where(seen, np.rint(np.ldexp(xd, q)), 0.0).astype(np.int64)
    keep = first[-w:] if first.size > w else first
    return m, keep.astype(np.int64), R[keep].astype(np.int16)


def encode_sequential(x, w: int):
    """The same, one entry at a time (a loop over the entries in the order
    of Sec. 6.1.3); for small inputs."""
    x = [float(v) for v in np.asarray(x).reshape(-1)]
    m, starts, exps = [], [], []
    run = None
    for i, v in enumerate(x):
        a = abs(v)
        if a != 0.0:
            _, e = np.frexp(a)
            e = int(e)
            if np.rint(np.ldexp(a, (w - 1) - e)) == float(1 << (w - 1)):
                e += 1
            if run is None or e > run:
                run = e
                starts.append(i)
                exps.append(e)
        m.append(0 if run is None else int(np.rint(np.ldexp(v, (w - 1) - run))))
    starts, exps = starts[-w:], exps[-w:]
    return np.array(m, dtype=np.int64), np.array(starts, dtype=np.int64), np.array(exps, dtype=np.int16)


def decode(m: np.ndarray, starts: np.ndarray, exps: np.ndarray, w: int, n: int | None = None) -> np.ndarray:
    """Float64 values: entry ``i`` takes the exponent of the last kept block
    starting at or before ``i``; entries before the first kept block are 0."""
    m = np.asarray(m, dtype=np.int64).reshape(-1)
    if n is not None:
        m = m[:n]
    starts = np.asarray(starts, dtype=np.int64)
    exps = np.asarray(exps, dtype=np.int64)
    out = np.zeros(m.size, dtype=np.float64)
    if starts.size == 0:
        return out
    k = np.searchsorted(starts, np.arange(m.size), side="right") - 1
    live = k >= 0
    q = exps[np.where(live, k, 0)] - (w - 1)
    out[live] = np.ldexp(m[live].astype(np.float64), q[live])
    return out


def storage_bytes(n: int, w: int, nblocks: int) -> int:
    """Codes (in the container of width ``w``) plus 10 bytes per kept block."""
    return n * bfp.container_bits(w) // 8 + 10 * nblocks
