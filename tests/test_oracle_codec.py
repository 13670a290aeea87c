"""Pins of the oracle's BFP codec (no GPU).

Checked against hand-derived cases (``tests/golden/bfp_examples.json``),
brute force over every code of small widths, the rounding error bound of
round-to-nearest, ties-to-even, idempotence, and the value-exactness of
widening (paper Sec. 4: increasing precision appends zero bits).
"""
import json
import os

import numpy as np
import pytest

from oracle import bfp

HERE = os.path.dirname(__file__)


def _golden():
    with open(os.path.join(HERE, "golden", "bfp_examples.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_hand_derived_cases(case):
    B, w = case["block"], case["w"]
    x = np.zeros(B)
    x[: len(case["x"])] = case["x"]
    m, e = bfp.encode(x, B, w)
    assert int(e[0]) == case["e"]
    assert list(m[: len(case["m"])]) == case["m"]
    assert not np.any(m[len(case["m"]):])
    d = bfp.decode(m, e, B, w)
    assert list(d[: len(case["decoded"])]) == case["decoded"]


@pytest.mark.parametrize("w", [2, 3, 4, 8, 12, 16])
def test_every_code_round_trips(w):
    lim = (1 << (w - 1)) - 1
    codes = np.arange(-lim, lim + 1, dtype=np.int64)
    B = 64
    pad = (-codes.size) % B
    codes = np.concatenate([codes, np.zeros(pad, dtype=np.int64)])
    blocks = codes.reshape(-1, B)
    # give every block its max so that the exponent is the one we choose
    blocks[:, 0] = lim
    for e0 in (-20, 0, 7):
        e = np.full(blocks.shape[0], e0, dtype=np.int16)
        x = bfp.decode(blocks.reshape(-1), e, B, w)
        m2, e2 = bfp.encode(x, B, w)
        assert np.array_equal(m2, blocks.reshape(-1))
        if lim >= 1 << (w - 2):      # max in [2**(w-2), 2**(w-1)) keeps the exponent
            assert np.all(e2 == e0)


@pytest.mark.parametrize("w", [3, 8, 12, 16, 24, 40, 53])
@pytest.mark.parametrize("B", [32, 64])
def test_error_bound_and_idempotence(w, B):
    rng = np.random.default_rng(w * 100 + B)
    x = rng.standard_normal(5 * B + 7) * np.exp(rng.uniform(-30, 30, 5 * B + 7))
    m, e = bfp.encode(x, B, w)
    assert m.size == 6 * B and e.size == 6
    lim = (1 << (w - 1)) - 1
    assert np.all(np.abs(m) <= lim)
    d = bfp.decode(m, e, B, w, x.size)
    q = np.repeat(e.astype(np.int64) - (w - 1), B)[: x.size]
    assert np.all(np.abs(x - d) <= np.ldexp(0.5, q))
    m2, e2 = bfp.encode(d, B, w)
    assert np.array_equal(m, m2) and np.array_equal(e, e2)


def test_float32_input_matches_float64_path():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(640).astype(np.float32)
    for w in (8, 12, 16, 24):
        a = bfp.encode(x, 64, w)
        b = bfp.encode(x.astype(np.float64), 64, w)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_ties_to_even_explicit():
    # a block whose max fixes q = 0 at w = 8 (max 100 -> e = 7, q = 0)
    x = np.zeros(32)
    x[:6] = [100.0, 2.5, 3.5, -2.5, -3.5, 0.5]
    m, e = bfp.encode(x, 32, 8)
    assert int(e[0]) == 7
    assert list(m[:6]) == [100, 2, 4, -2, -4, 0]


def test_denormal_and_tiny_inputs():
    x = np.zeros(64)
    x[0] = 5e-324
    x[1] = -2.5e-310
    m, e = bfp.encode(x, 64, 16)
    d = bfp.decode(m, e, 64, 16)
    q = int(e[0]) - 15
    assert abs(d[1] - x[1]) <= np.ldexp(0.5, q)
    assert d[0] == 0.0


def test_nonfinite_rejected():
    with pytest.raises(ValueError):
        bfp.encode(np.array([1.0, np.nan]), 32, 8)
    with pytest.raises(ValueError):
        bfp.encode(np.array([np.inf]), 32, 8)


@pytest.mark.parametrize("w,k", [(4, 2), (8, 1), (12, 4), (16, 16), (30, 23)])
def test_widening_is_exact_reencoding(w, k):
    rng = np.random.default_rng(w + k)
    x = rng.standard_normal(256) * 3.0
    m, e = bfp.encode(x, 64, w)
    wide = bfp.widen(m, k)
    assert np.array_equal(bfp.decode(wide, e, 64, w + k), bfp.decode(m, e, 64, w))
    m2, e2 = bfp.encode(bfp.decode(m, e, 64, w), 64, w + k)
    assert np.array_equal(m2, wide) and np.array_equal(e2, e)


@pytest.mark.parametrize("w", [4, 8, 11, 12, 13, 16, 20, 32, 33, 53])
def test_pack_unpack(w):
    rng = np.random.default_rng(w)
    lim = (1 << (w - 1)) - 1
    m = rng.integers(-lim, lim + 1, size=128)
    buf = bfp.pack(m, w)
    assert len(buf) == 128 * bfp.container_bits(w) // 8
    assert np.array_equal(bfp.unpack(buf, w, 128), m)


def test_twelve_bit_layout():
    # value t occupies bits 12t..12t+11, little endian
    buf = bfp.pack(np.array([0x123, -1]), 12)
    assert buf == bytes([0x23, 0xF1, 0xFF])
