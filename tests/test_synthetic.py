"""The seeded input generators (no GPU): shapes, boundary values,
statistics, and bit-identity of the numpy and torch hash-noise builders."""
import numpy as np

import synthetic as S


def test_sine_rhs_shape_and_boundary():
    f = S.sine_rhs(3, 4)
    assert f.shape == (17, 17, 17)
    assert not np.any(f[0]) and not np.any(f[-1]) and not np.any(f[:, :, 0])
    assert np.isclose(f[8, 8, 8], 3 * np.pi ** 2)


def test_splitmix_reference_values():
    # SplitMix64 from state 0: the first outputs of the published generator
    # (Vigna's splitmix64.c seeded with 0) are 0xe220a8397b1dcdaf,
    # 0x6e789e6aa1b965f4; counter i uses state i*gamma after one increment.
    import numpy as np
    u = S.splitmix64_uniform(0, np.array([0], dtype=np.int64))
    assert u[0] == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


def test_hash_noise_numpy_torch_identical():
    import torch
    a = S.hash_noise_rhs(3, 4, amp=1e-4, seed=3)
    b = S.hash_noise_rhs_torch(3, 4, amp=1e-4, seed=3).numpy()
    assert np.array_equal(a, b)
    noise = a - S.sine_rhs(3, 4)
    assert np.abs(noise).max() <= 1e-4 and np.abs(noise).max() > 0.9e-4
    assert not np.any(noise[0])


def test_gaussian_field_statistics():
    g = S.gaussian_random_field(3, 32, 0.1, 1)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    # correlated: neighbours are strongly correlated at corr length 0.1 (3.2 cells)
    c = np.corrcoef(g[:, :, :-1].ravel(), g[:, :, 1:].ravel())[0, 1]
    assert 0.8 < c < 1.0


def test_smoothed_rhs_unit_std():
    f = S.smoothed_noise_rhs(3, 4, 100)
    assert np.isclose(f[1:-1, 1:-1, 1:-1].std(), 1.0)
    assert not np.any(f[0])


def test_torch_smoothing_matches_numpy_on_the_same_noise():
    import torch
    dim, L, seed = 3, 4, 21
    N = (1 << L) + 1
    w = np.random.default_rng(seed).standard_normal(((N - 2),) * dim)
    ref = S.smoothed_noise_rhs(dim, L, seed)
    got = S._smooth_torch(torch.from_numpy(w), dim, 4).numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    f = S.smoothed_noise_rhs_torch(dim, L, seed)
    assert f.shape == (N,) * dim and float(f[0].abs().max()) == 0.0
    assert abs(float(f[1:-1, 1:-1, 1:-1].std(unbiased=False)) - 1.0) < 1e-12


def test_torch_random_field_matches_numpy_on_the_same_noise():
    import torch
    dim, ncell, corr, seed = 3, 16, 0.2, 5
    w = np.random.default_rng(seed).standard_normal((ncell,) * dim)
    ref = S.gaussian_random_field(dim, ncell, corr, seed)
    got = S._grf_filter_torch(torch.from_numpy(w), corr).numpy()
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-12)
    k = S.lognormal_kappa_torch(dim, 4, corr, seed)
    assert k.shape == (16, 16, 16) and float(k.min()) > 0.0
