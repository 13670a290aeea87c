"""Pins of the oracle's adaptive-exponent BFP codec (no GPU).

Sec. 6.1.3 (Exponents): running-maximum exponents, a new block where the
exponent rises, only the ``w`` largest exponents kept.  Pinned against
hand-derived cases (``tests/golden/adaptive_bfp_examples.json``), a
one-entry-at-a-time loop, the already pinned fixed-block codec (a vector
whose largest exponent comes first is a single block), the paper's claim
that dropped entries round to zero in scaled fixed point, the half-quantum
error bound, and nesting of the quantisation grids (never less accurate
than single-exponent BFP).
"""
import json
import os

import numpy as np
import pytest

from oracle import adaptive, bfp

HERE = os.path.dirname(__file__)


def _golden():
    with open(os.path.join(HERE, "golden", "adaptive_bfp_examples.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_hand_derived_cases(case):
    w = case["w"]
    m, s, e = adaptive.encode(np.array(case["x"]), w)
    assert list(m) == case["m"]
    assert list(s) == case["starts"]
    assert list(e) == case["exps"]
    assert list(adaptive.decode(m, s, e, w)) == case["decoded"]


def _vectors(rng, n):
    """Magnitudes spread over many binades, rising trends, zeros, ties."""
    yield rng.standard_normal(n)
    yield rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n))
    yield np.exp2(np.linspace(-60, 60, n)) * rng.choice([-1.0, 1.0], n)   # many rising exponents
    z = rng.standard_normal(n)
    z[: n // 3] = 0.0
    z[rng.random(n) < 0.2] = 0.0
    yield z
    yield np.round(rng.standard_normal(n) * 8) / 4                         # exact binary ties
    yield rng.standard_normal(n).astype(np.float32)


@pytest.mark.parametrize("w", [2, 3, 5, 8, 12, 16, 24, 31, 53])
def test_vectorised_equals_entry_by_entry_loop(w):
    rng = np.random.default_rng(w)
    for x in _vectors(rng, 300):
        a = adaptive.encode(x, w)
        b = adaptive.encode_sequential(x, w)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


@pytest.mark.parametrize("w", [3, 8, 16, 30])
@pytest.mark.parametrize("B", [32, 64])
def test_largest_first_is_one_fixed_block(w, B):
    """The largest exponent first: one block, the fixed-block codes."""
    rng = np.random.default_rng(7 * w + B)
    x = rng.standard_normal(B)
    x[0] = 1.5 * np.max(np.abs(x))
    m, s, e = adaptive.encode(x, w)
    mf, ef = bfp.encode(x, B, w)
    assert list(s) == [0] and int(e[0]) == int(ef[0])
    assert np.array_equal(m, mf)


@pytest.mark.parametrize("w", [2, 4, 8, 16, 40])
def test_error_bounds_and_scaled_fixed_point(w):
    rng = np.random.default_rng(100 + w)
    for x in _vectors(rng, 64):
        x = np.asarray(x, dtype=np.float64)
        m, s, e = adaptive.encode(x, w)
        d = adaptive.decode(m, s, e, w)
        lim = (1 << (w - 1)) - 1
        assert np.all(np.abs(m) <= lim)
        if not np.any(x):
            assert s.size == 0 and not np.any(d)
            continue
        # running exponent of each entry, and the first kept entry
        R = np.maximum.accumulate(adaptive.entry_exponents(x, w))
        first = int(s[0])
        kept = np.arange(x.size) >= first
        # kept entries: within half a quantum of their block
        assert np.all(np.abs(x - d)[kept] <= np.ldexp(1.0, R[kept] - w))
        # dropped entries decode to 0 and would round to 0 in scaled fixed
        # point (one exponent for the 64 values), as the paper argues
        assert not np.any(d[~kept])
        mf, ef = bfp.encode(x, 64, w)
        assert not np.any(mf[: x.size][~kept])
        # nested power-of-two grids: never less accurate than one exponent
        df = bfp.decode(mf, ef, 64, w, n=x.size)
        assert np.all(np.abs(x - d) <= np.abs(x - df))
        assert len(s) <= w and np.all(np.diff(s) > 0) and np.all(np.diff(e.astype(int)) > 0)


@pytest.mark.parametrize("w", [3, 8, 16])
def test_decode_encode_is_stable(w):
    rng = np.random.default_rng(5 + w)
    for x in _vectors(rng, 200):
        m, s, e = adaptive.encode(x, w)
        d = adaptive.decode(m, s, e, w)
        m2, s2, e2 = adaptive.encode(d, w)
        assert np.array_equal(adaptive.decode(m2, s2, e2, w), d)


def test_rejects_non_finite():
    with pytest.raises(ValueError):
        adaptive.encode(np.array([1.0, np.inf]), 8)
