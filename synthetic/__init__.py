"""Seeded synthetic inputs for the compact-multigrid workloads.

This module only *makes inputs*: right-hand sides, noise, diffusion
coefficient fields and manufactured solutions.  It contains none of the
solver's arithmetic, so both the CPU oracle and the GPU library can take
their inputs from here without sharing any method code.

Conventions (the same as the public C ABI):

* A problem on the unit square/cube with finest level ``L`` has
  ``N = 2**L + 1`` nodes per axis; node ``i`` sits at ``x = i / 2**L``.
* Node arrays have shape ``(N,)*dim`` in C order with ``x`` fastest, i.e.
  index order ``[z, y, x]`` in 3-D and ``[y, x]`` in 2-D.
* Cell arrays (diffusion coefficient) have shape ``(2**L,)*dim``; cell
  ``c`` spans nodes ``c .. c+1`` on every axis.

The manufactured solution is the one the workloads name: the product of
``sin(pi x_i)``; its right-hand side for ``-Laplace u = f`` is
``dim * pi**2 * u``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "nodes_1d", "sine_solution", "sine_rhs", "gaussian_noise_rhs",
    "splitmix64_uniform", "splitmix64_uniform_torch", "hash_noise_rhs",
    "hash_noise_rhs_torch", "gaussian_random_field", "lognormal_kappa",
    "smoothed_noise_rhs", "exponent_mix", "WORKLOADS",
]


def nodes_1d(L: int) -> np.ndarray:
    """Node coordinates ``i / 2**L`` for ``i = 0 .. 2**L`` (exact in binary)."""
    n = 1 << L
    return np.arange(n + 1, dtype=np.float64) / float(n)


def _sin_pi(L: int) -> np.ndarray:
    s = np.sin(np.pi * nodes_1d(L))
    s[0] = 0.0
    s[-1] = 0.0  # sin(pi) is 1.2e-16 in floating point; the boundary is exactly 0
    return s


def sine_solution(dim: int, L: int) -> np.ndarray:
    """``u*(x) = prod_i sin(pi x_i)`` sampled on the ``N**dim`` node grid."""
    s = _sin_pi(L)
    if dim == 2:
        return np.multiply.outer(s, s)
    if dim == 3:
        return np.multiply.outer(np.multiply.outer(s, s), s)
    raise ValueError("dim must be 2 or 3")


def sine_rhs(dim: int, L: int) -> np.ndarray:
    """``f = dim * pi**2 * u*``: the right-hand side of ``-Laplace u* = f``."""
    return (dim * np.pi ** 2) * sine_solution(dim, L)


def gaussian_noise_rhs(dim: int, L: int, sigma: float = 1e-3, seed: int = 0) -> np.ndarray:
    """Sine right-hand side plus ``sigma * N(0, 1)`` on the interior nodes.

    The normal draws come from ``numpy.random.default_rng(seed)`` in C order
    over the interior nodes (boundary nodes get no noise).
    """
    f = sine_rhs(dim, L)
    m = (1 << L) - 1
    noise = np.random.default_rng(seed).standard_normal((m,) * dim)
    f[(slice(1, -1),) * dim] += sigma * noise
    return f


# --------------------------------------------------------------------------
# Counter-based uniform noise (SplitMix64, Steele, Lea & Flood, OOPSLA 2014)
# --------------------------------------------------------------------------
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def splitmix64_uniform(seed: int, index: np.ndarray) -> np.ndarray:
    """Uniform ``[0, 1)`` doubles from the SplitMix64 output function.

    The state for counter ``i`` is ``seed * 2**40 + i`` advanced by one
    golden-ratio increment; the 64-bit finaliser (xor-shift 30/27/31 with the
    two published multipliers) mixes it and the top 53 bits give the double.
    """
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) << np.uint64(40)) + index.astype(np.uint64)
        z = z + np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _as_i64(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


def splitmix64_uniform_torch(seed: int, index):
    """The same generator on a torch int64 tensor (any device), bit-identical.

    torch has no unsigned 64-bit arithmetic, so the logical right shifts are
    written as arithmetic shifts followed by a mask; products wrap modulo
    ``2**64`` exactly as the unsigned ones do.
    """
    import torch

    def lsr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    z = index.to(torch.int64) + (seed << 40)
    z = z + _as_i64(_GAMMA)
    z = (z ^ lsr(z, 30)) * _as_i64(_M1)
    z = (z ^ lsr(z, 27)) * _as_i64(_M2)
    z = z ^ lsr(z, 31)
    return lsr(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def hash_noise_rhs(dim: int, L: int, amp: float = 1e-4, seed: int = 3) -> np.ndarray:
    """Sine right-hand side plus ``amp * U[-1, 1)`` hashed from the node index.

    The counter is the linear C-order index of the node in the ``N**dim``
    array; boundary nodes get no noise.  Built plane by plane to bound memory.
    """
    f = sine_rhs(dim, L)
    N = (1 << L) + 1
    plane = N ** (dim - 1)
    inner = (slice(1, -1),) * (dim - 1)
    for k in range(1, N - 1):
        idx = np.arange(k * plane, (k + 1) * plane, dtype=np.int64).reshape((N,) * (dim - 1))
        u = splitmix64_uniform(seed, idx)
        f[k][inner] += amp * (2.0 * u[inner] - 1.0)
    return f


def hash_noise_rhs_torch(dim: int, L: int, amp: float = 1e-4, seed: int = 3, device="cpu"):
    """:func:`hash_noise_rhs` built directly on a torch device (bit-identical).

    The sine factor is formed from the same float64 1-D sample vector and the
    same product order (``(s_z * s_y) * s_x``), so the result matches the
    numpy version exactly.
    """
    import torch

    s = torch.from_numpy(_sin_pi(L)).to(device)
    N = (1 << L) + 1
    if dim == 2:
        base = s[:, None] * s[None, :]
    else:
        base = (s[:, None, None] * s[None, :, None]) * s[None, None, :]
    f = (dim * np.pi ** 2) * base
    plane = N ** (dim - 1)
    inner = (slice(1, -1),) * (dim - 1)
    for k in range(1, N - 1):
        idx = torch.arange(k * plane, (k + 1) * plane, dtype=torch.int64, device=device)
        u = splitmix64_uniform_torch(seed, idx).reshape((N,) * (dim - 1))
        f[k][inner] += amp * (2.0 * u[inner] - 1.0)
    return f


# --------------------------------------------------------------------------
# Random diffusion coefficients and smoothed random right-hand sides
# --------------------------------------------------------------------------
def gaussian_random_field(dim: int, ncell: int, corr_len: float, seed: int) -> np.ndarray:
    """Zero-mean, unit-sample-variance field with Gaussian covariance.

    Spectral synthesis on the periodic ``ncell**dim`` cell grid of the unit
    cube: white noise from ``default_rng(seed)`` is filtered in Fourier space
    by the square root of the spectral density ``exp(-|k|^2 l^2 / 2)`` of the
    covariance ``exp(-r^2 / (2 l^2))`` and then standardised.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ncell,) * dim)
    wh = np.fft.rfftn(w)
    h = 1.0 / ncell
    k_full = 2.0 * np.pi * np.fft.fftfreq(ncell, d=h)
    k_half = 2.0 * np.pi * np.fft.rfftfreq(ncell, d=h)
    axes = [k_full] * (dim - 1) + [k_half]
    k2 = np.zeros(wh.shape)
    for ax, k in enumerate(axes):
        shape = [1] * dim
        shape[ax] = k.size
        k2 = k2 + (k.reshape(shape)) ** 2
    wh *= np.exp(-0.25 * k2 * corr_len ** 2)
    g = np.fft.irfftn(wh, s=(ncell,) * dim, axes=tuple(range(dim)))
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_kappa(dim: int, L: int, corr_len: float, seed: int) -> np.ndarray:
    """Cell coefficient ``kappa = exp(G)`` on the ``(2**L)**dim`` cells."""
    return np.exp(gaussian_random_field(dim, 1 << L, corr_len, seed))


def smoothed_noise_rhs(dim: int, L: int, seed: int, passes: int = 4) -> np.ndarray:
    """White ``N(0, 1)`` on interior nodes, smoothed and rescaled.

    Each pass applies the separable ``[1, 2, 1] / 4`` filter along every axis
    with zero Dirichlet nodes; the result is rescaled to unit sample standard
    deviation over the interior.
    """
    N = (1 << L) + 1
    f = np.zeros((N,) * dim)
    inner = (slice(1, -1),) * dim
    f[inner] = np.random.default_rng(seed).standard_normal(((N - 2),) * dim)
    for _ in range(passes):
        for ax in range(dim):
            g = np.zeros_like(f)
            lo = [slice(1, -1)] * dim
            mid = [slice(1, -1)] * dim
            hi = [slice(1, -1)] * dim
            lo[ax] = slice(0, -2)
            hi[ax] = slice(2, None)
            g[inner] = 0.25 * f[tuple(lo)] + 0.5 * f[tuple(mid)] + 0.25 * f[tuple(hi)]
            f = g
    f[inner] /= f[inner].std()
    return f


def _smooth_torch(w, dim: int, passes: int):
    """The filter and rescaling of :func:`smoothed_noise_rhs` on a torch
    tensor ``w`` of interior white noise (same operation order per node)."""
    import torch
    N = w.shape[0] + 2
    f = torch.zeros((N,) * dim, dtype=torch.float64, device=w.device)
    inner = (slice(1, -1),) * dim
    f[inner] = w
    for _ in range(passes):
        for ax in range(dim):
            g = torch.zeros_like(f)
            lo = [slice(1, -1)] * dim
            mid = [slice(1, -1)] * dim
            hi = [slice(1, -1)] * dim
            lo[ax] = slice(0, -2)
            hi[ax] = slice(2, None)
            g[inner] = 0.25 * f[tuple(lo)] + 0.5 * f[tuple(mid)] + 0.25 * f[tuple(hi)]
            f = g
    f[inner] /= f[inner].std(unbiased=False)
    return f


def smoothed_noise_rhs_torch(dim: int, L: int, seed: int, passes: int = 4, device="cpu"):
    """:func:`smoothed_noise_rhs` built on a torch device for large grids.

    The white noise comes from ``torch.Generator(device).manual_seed(seed)``
    (so the draws, unlike the filter, depend on the device type).
    """
    import torch
    N = (1 << L) + 1
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    w = torch.randn(((N - 2),) * dim, generator=gen, dtype=torch.float64, device=device)
    return _smooth_torch(w, dim, passes)


def _grf_filter_torch(w, corr_len: float):
    """The spectral filter and standardisation of
    :func:`gaussian_random_field` applied to white noise ``w``."""
    import torch
    dim, ncell = w.dim(), w.shape[0]
    wh = torch.fft.rfftn(w)
    k_full = 2.0 * np.pi * torch.fft.fftfreq(ncell, d=1.0 / ncell, dtype=torch.float64, device=w.device)
    k_half = 2.0 * np.pi * torch.fft.rfftfreq(ncell, d=1.0 / ncell, dtype=torch.float64, device=w.device)
    axes = [k_full] * (dim - 1) + [k_half]
    k2 = torch.zeros(wh.shape, dtype=torch.float64, device=w.device)
    for ax, k in enumerate(axes):
        shape = [1] * dim
        shape[ax] = k.numel()
        k2 = k2 + k.reshape(shape) ** 2
    wh = wh * torch.exp(-0.25 * k2 * corr_len ** 2)
    g = torch.fft.irfftn(wh, s=(ncell,) * dim)
    g = g - g.mean()
    return g / g.std(unbiased=False)


def lognormal_kappa_torch(dim: int, L: int, corr_len: float, seed: int, device="cpu"):
    """:func:`lognormal_kappa` built on a torch device for large grids (white
    noise from ``torch.Generator(device).manual_seed(seed)``)."""
    import torch
    ncell = 1 << L
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    w = torch.randn((ncell,) * dim, generator=gen, dtype=torch.float64, device=device)
    return torch.exp(_grf_filter_torch(w, corr_len))


# The five workloads (problem shape, inputs and solver settings).
WORKLOADS = {
    "poisson2d_129": dict(dim=2, L=7, op="poisson", smoother="wjacobi", omega=0.8,
                          nu_pre=2, nu_post=2, ir_iters=2, bfp_block=32, bits=16,
                          rhs="gaussian_noise", sigma=1e-3, seed=0),
    "poisson3d_257": dict(dim=3, L=8, op="poisson", smoother="rbgs", omega=1.0,
                          nu_pre=2, nu_post=2, ir_iters=2, bfp_block=64, bits=(8, 12, 16),
                          rhs="sine"),
    "poisson3d_1025": dict(dim=3, L=10, op="poisson", smoother="rbgs", omega=1.0,
                           nu_pre=2, nu_post=2, ir_iters=2, bfp_block=64, bits=(8, 12, 16),
                           rhs="hash_noise", amp=1e-4, seed=3),
    # diffusion: N = 3, the smallest N whose error against the converged
    # solve stays below half the Richardson estimate of the discretisation
    # error on both problems (N = 2 reaches 0.65x on the 129^3 problem)
    "diffusion3d_129": dict(dim=3, L=7, op="diffusion", smoother="rbgs", omega=1.0,
                            nu_pre=2, nu_post=2, ir_iters=3, bfp_block=64, bits=16,
                            kappa_corr=0.1, kappa_seed=1, kappa_obs_seed=2, rhs="ones"),
    "diffusion3d_513x8": dict(dim=3, L=9, op="diffusion", smoother="rbgs", omega=1.0,
                              nu_pre=2, nu_post=2, ir_iters=3, bfp_block=64, bits=16,
                              kappa_corr=0.05, kappa_seed=4, kappa_obs_seed=5,
                              rhs="smoothed_noise", rhs_seeds=tuple(range(100, 108))),
}


# ------------------------------------------------------ codec test vectors
EXPONENT_MIX_KINDS = ("normal", "binades", "rising", "zeros", "ties", "float32")


def exponent_mix(n: int, kind: str, seed: int) -> np.ndarray:
    """Seeded vectors for codec tests, with magnitudes that exercise block
    exponents: ``normal`` N(0,1); ``binades`` N(0,1) scaled by 2**k, k
    uniform in [-40, 40); ``rising`` magnitudes 2**-60 .. 2**60 in order
    (a new exponent every few entries) with random signs; ``zeros`` N(0,1)
    with a leading third and a fifth of the rest zero; ``ties`` multiples of
    1/4 (exact binary ties); ``float32`` N(0,1) as float32."""
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(n)
    if kind == "binades":
        return rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n).astype(np.float64))
    if kind == "rising":
        return np.exp2(np.linspace(-60.0, 60.0, n)) * rng.choice([-1.0, 1.0], n)
    if kind == "zeros":
        z = rng.standard_normal(n)
        z[: n // 3] = 0.0
        z[rng.random(n) < 0.2] = 0.0
        return z
    if kind == "ties":
        return np.round(rng.standard_normal(n) * 8.0) / 4.0
    if kind == "float32":
        return rng.standard_normal(n).astype(np.float32)
    raise ValueError(kind)
