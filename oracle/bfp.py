"""Block floating point (BFP) codec — oracle (test infrastructure only).

The paper stores the compact sections, residual and correction in BFP
format: one shared exponent for a block of mantissas (Sec. 6.1.3,
"Exponents").  Decreasing precision rounds to the nearest representable
value with ties to even; increasing precision appends zero bits (Sec. 4,
the precision-change rule under Table 1).  The bit counts include the sign
(caption of Table 2).

Readings fixed here (the paper does not pin them down):

* blocks are ``B`` consecutive values of the padded level array (B = 32 or 64),
  the tail block padded with zeros;
* block exponent ``e`` is the ``frexp`` exponent of the block's largest
  magnitude (``2**(e-1) <= max|x| < 2**e``); the quantum is
  ``q = e - (w - 1)`` and mantissas are ``m = RNE(x * 2**-q)``;
* if rounding the largest magnitude reaches ``2**(w-1)`` the exponent is
  raised by one and the block re-rounded, so mantissas always lie in
  ``[-(2**(w-1) - 1), 2**(w-1) - 1]`` (symmetric two's complement);
* an all-zero block stores the sentinel exponent ``-32768`` and zero codes;
* non-finite input is an error.

Storage containers: ``w <= 8`` int8, ``<= 12`` packed 12-bit (two values in
three bytes, value ``t`` at bit ``12 t``, little endian), ``<= 16`` int16,
``<= 32`` int32, ``<= 53`` int64, each sign-extended.
"""
from __future__ import annotations

import numpy as np

ZERO_EXP = -32768
MAX_BITS = 53


def container_bits(w: int) -> int:
    """Container width (bits) that stores a ``w``-bit code."""
    if not 2 <= w <= MAX_BITS:
        raise ValueError(f"width {w} outside [2, {MAX_BITS}]")
    for c in (8, 12, 16, 32):
        if w <= c:
            return c
    return 64


def n_blocks(n: int, B: int) -> int:
    return (n + B - 1) // B


def encode(x: np.ndarray, B: int, w: int):
    """Quantise the flat array ``x`` to ``w``-bit BFP with blocks of ``B``.

    Returns ``(m, e)``: int64 mantissas of length ``n_blocks * B`` (padding
    included) and int16 block exponents.  ``x`` may be float32 or float64;
    both are widened to float64 exactly before rounding.
    """
    if B not in (32, 64):
        raise ValueError("block must be 32 or 64")
    container_bits(w)
    x = np.asarray(x).reshape(-1)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite value in BFP input")
    nb = n_blocks(x.size, B)
    xb = np.zeros(nb * B, dtype=np.float64)
    xb[: x.size] = x.astype(np.float64)
    xb = xb.reshape(nb, B)
    a = np.max(np.abs(xb), axis=1)
    zero = a == 0.0
    _, e = np.frexp(a)                     # a = f * 2**e, 0.5 <= f < 1
    e = e.astype(np.int64)
    q = e - (w - 1)
    top = np.rint(np.ldexp(a, -q))         # largest magnitude in units of 2**q
    bump = (~zero) & (top == float(1 << (w - 1)))
    e = np.where(bump, e + 1, e)
    q = e - (w - 1)
    m = np.rint(np.ldexp(xb, -q[:, None])).astype(np.int64)
    m[zero] = 0
    e = np.where(zero, ZERO_EXP, e)
    return m.reshape(-1), e.astype(np.int16)


def decode(m: np.ndarray, e: np.ndarray, B: int, w: int, n: int | None = None,
           dtype=np.float64) -> np.ndarray:
    """Values ``m * 2**(e - (w - 1))``; exact in float64 for ``w <= 53``.

    A float32 result is the round-to-nearest-even cast of the float64 value.
    """
    m = np.asarray(m, dtype=np.int64).reshape(-1, B)
    e = np.asarray(e, dtype=np.int64)
    q = e - (w - 1)
    q = np.where(e == ZERO_EXP, 0, q)
    x = np.ldexp(m.astype(np.float64), q[:, None]).reshape(-1)
    if n is not None:
        x = x[:n]
    return x.astype(dtype)


def widen(m: np.ndarray, k: int) -> np.ndarray:
    """Raise the width of a section by ``k`` bits: append ``k`` zero bits.

    The exponent ``e`` is unchanged (the quantum drops by ``k``); the value of
    every entry is unchanged (Sec. 2.2, prolongating a compact vector;
    Sec. 4, increasing precision).
    """
    return np.asarray(m, dtype=np.int64) * (1 << k)


# ------------------------------------------------------------------ packing
def pack(m: np.ndarray, w: int) -> bytes:
    """Pack int64 codes into the container of width ``container_bits(w)``."""
    c = container_bits(w)
    m = np.asarray(m, dtype=np.int64)
    lim = 1 << (w - 1)
    if m.size and (m.max() >= lim or m.min() <= -lim):
        raise ValueError("code outside the width")
    if c == 8:
        return m.astype(np.int8).tobytes()
    if c == 16:
        return m.astype(np.int16).tobytes()
    if c == 32:
        return m.astype(np.int32).tobytes()
    if c == 64:
        return m.astype(np.int64).tobytes()
    # 12-bit: value t occupies bits 12t .. 12t+11 of a little-endian stream
    if m.size % 2:
        raise ValueError("12-bit packing needs an even count")
    u = (m & 0xFFF).astype(np.uint32).reshape(-1, 2)
    word = u[:, 0] | (u[:, 1] << 12)          # 24 bits per pair
    out = np.empty((u.shape[0], 3), dtype=np.uint8)
    out[:, 0] = word & 0xFF
    out[:, 1] = (word >> 8) & 0xFF
    out[:, 2] = (word >> 16) & 0xFF
    return out.tobytes()


def unpack(buf: bytes, w: int, count: int) -> np.ndarray:
    """Inverse of :func:`pack` (sign-extends to int64)."""
    c = container_bits(w)
    if c == 8:
        return np.frombuffer(buf, dtype=np.int8, count=count).astype(np.int64)
    if c == 16:
        return np.frombuffer(buf, dtype=np.int16, count=count).astype(np.int64)
    if c == 32:
        return np.frombuffer(buf, dtype=np.int32, count=count).astype(np.int64)
    if c == 64:
        return np.frombuffer(buf, dtype=np.int64, count=count).astype(np.int64)
    b = np.frombuffer(buf, dtype=np.uint8, count=count * 3 // 2).astype(np.int64).reshape(-1, 3)
    word = b[:, 0] | (b[:, 1] << 8) | (b[:, 2] << 16)
    v = np.stack([word & 0xFFF, (word >> 12) & 0xFFF], axis=1).reshape(-1)
    return np.where(v >= 2048, v - 4096, v)


def storage_bytes(n: int, B: int, w: int) -> int:
    """Bytes of one stored section: packed codes plus one int16 per block."""
    nb = n_blocks(n, B)
    return nb * B * container_bits(w) // 8 + 2 * nb
