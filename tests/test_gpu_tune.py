"""Tuning of the precision constants (Sec. 7.1) with the library's solver:
the GPU search selects exactly the widths and iteration count that the
oracle's search selects (the solves are bit-identical, so every acceptance
decision is the same)."""
import pytest

from oracle import tune as otune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,Lmax,opts,ocfg", [
    (2, 5, dict(smoother="wjacobi", omega=0.8, bfp_block=32), dict(smoother="wjacobi", omega=0.8, block=32)),
    (3, 5, dict(smoother="rbgs", omega=1.0, bfp_block=64), dict(smoother="rbgs", omega=1.0, block=64)),
])
def test_gpu_tuning_matches_oracle(gpu_lib, dim, Lmax, opts, ocfg):
    from paper_2511_19036_amd.tune import tune_widths
    got = tune_widths(dim, Lmax, **opts)
    assert got == otune.tune(dim, Lmax, **ocfg)
