"""The oracle's tuning of the precision constants (Sec. 7.1) — no GPU.

Pins: the discretisation error it measures against equals the closed form
``(c_h - 1) ||u*||_h`` with ``||u*||_h = 2^(-d/2)`` (the discrete sum of
``sin^2`` over the grid is exact); generous settings pass and a 2-bit
residual fails; and the incremental search returns what an exhaustive
evaluation of the acceptance test over every candidate value selects.
"""
import numpy as np
import pytest

from oracle import tune

CFG2 = dict(smoother="wjacobi", omega=0.8, block=32)


def test_discretisation_error_closed_form():
    for dim, L in [(2, 4), (3, 3)]:
        e = tune.errors(dim, L, 30, 20, 12, **(CFG2 if dim == 2 else dict(block=64)))
        h = 2.0 ** -L
        ch = ((np.pi * h / 2) / np.sin(np.pi * h / 2)) ** 2
        for lev, (_, disc) in e.items():
            hl = 2.0 ** -lev
            chl = ((np.pi * hl / 2) / np.sin(np.pi * hl / 2)) ** 2
            assert disc == pytest.approx((chl - 1.0) * 2.0 ** (-dim / 2), rel=1e-12)
        assert e[L][1] == pytest.approx((ch - 1.0) * 2.0 ** (-dim / 2), rel=1e-12)


def test_generous_settings_pass_and_two_bits_fail():
    assert tune.accepted(2, 3, 5, 30, 20, 12, **CFG2)
    assert not tune.accepted(2, 3, 5, 30, 2, 12, **CFG2)


def test_search_matches_exhaustive_evaluation():
    dim, Lmin, Lmax = 2, 3, 5
    got = tune.tune(dim, Lmax, Lmin, **CFG2)

    def pick(values, ok):
        passes = {v: ok(v) for v in values}
        for v in values[:-1]:
            if passes[v] and passes[v + 1]:
                return v + 1
        return None

    b2 = pick(list(range(2, 25)), lambda b: tune.accepted(dim, Lmin, Lmax, 30, b, 12, **CFG2))
    b1 = pick(list(range(2, 54)), lambda b: tune.accepted(dim, Lmin, Lmax, b, b2, 12, **CFG2))
    N = pick(list(range(1, 13)), lambda k: tune.accepted(dim, Lmin, Lmax, b1, b2, k, **CFG2))
    assert got == {"bits_u": b1, "bits_r": b2, "bits_y": b2, "ir_iters": N}
    # the selected setting passes, and the width below the selected residual width
    # is where the acceptance test starts to hold (one bit of margin)
    assert tune.accepted(dim, Lmin, Lmax, b1, b2, N, **CFG2)
