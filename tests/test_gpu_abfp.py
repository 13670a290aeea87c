"""GPU parity of the adaptive-exponent BFP codec (Sec. 6.1.3, Exponents).

The HIP encoder (one pass, decoupled look-back over tiles of 4096 values)
against the oracle: bit-exact codes, kept blocks and decoded values, over
widths 2..53, both input types, lengths around and across tile boundaries,
vectors with many rising exponents (blocks dropped), all-zero and leading
zero vectors, non-finite input, and a 2^27-value vector.
"""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import adaptive as oa
from oracle import bfp as ob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cmg(gpu_lib):
    import paper_2511_19036_amd
    return paper_2511_19036_amd


def _run(cmg, x, w):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    codes, starts, exps, nb = cmg.abfp_encode(xt, w)
    d = cmg.abfp_decode(codes, starts, exps, nb, x.size, w)
    torch.cuda.synchronize()
    k = int(nb.item())
    npad = (x.size + 63) // 64 * 64
    m = ob.unpack(codes.cpu().numpy().tobytes(), w, npad)
    return m, starts.cpu().numpy()[: max(k, 0)], exps.cpu().numpy()[: max(k, 0)], k, d.cpu().numpy()


def _check(cmg, x, w):
    m, s, e, k, d = _run(cmg, x, w)
    mo, so, eo = oa.encode(x, w)
    assert k == so.size
    assert np.array_equal(m[: x.size], mo), "codes"
    assert not np.any(m[x.size:]), "padding codes"
    assert np.array_equal(s, so) and np.array_equal(e, eo), "kept blocks"
    assert np.array_equal(d, oa.decode(mo, so, eo, w)), "decoded values"


@pytest.mark.parametrize("w", [2, 3, 5, 8, 11, 12, 16, 24, 31, 53])
@pytest.mark.parametrize("kind", S.EXPONENT_MIX_KINDS)
def test_abfp_bit_exact(cmg, w, kind):
    for n in (1, 17, 64, 4095, 4096, 4097, 3 * 4096 + 100):
        _check(cmg, S.exponent_mix(n, kind, seed=1000 * w + n), w)


@pytest.mark.parametrize("w", [4, 16])
def test_abfp_many_tiles(cmg, w):
    for kind in ("rising", "binades", "zeros"):
        _check(cmg, S.exponent_mix(200_003, kind, seed=w), w)


def test_abfp_degenerate(cmg):
    _check(cmg, np.zeros(5000), 16)                     # no block at all
    x = np.zeros(9000)
    x[8999] = -3.0                                      # the only block starts in the last tile
    _check(cmg, x, 8)
    x = np.zeros(70)
    _check(cmg, x[:0], 16)                              # empty vector


def test_abfp_nonfinite_reported(cmg):
    x = S.exponent_mix(10_000, "normal", seed=3)
    x[7777] = np.nan
    _, _, _, k, _ = _run(cmg, x, 12)
    assert k == -1


def test_abfp_large_vector(cmg):
    """2^27 values (a 513^3-sized vector): the whole result against the
    oracle, and the storage claim (codes plus at most w blocks)."""
    x = S.exponent_mix(1 << 27, "binades", seed=11)
    _check(cmg, x, 16)
    assert oa.storage_bytes(x.size, 16, 16) == 2 * x.size + 160
