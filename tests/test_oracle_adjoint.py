"""Pins of the oracle's adjoint gradient (no GPU).

Brute force on tiny grids: dense ``A(kappa)`` assembled edge by edge,
``u = A^-1 f``, ``lambda = A^-1 (u - u_obs)`` and
``dJ/dkappa_c = -lambda^T (dA/dkappa_c) u`` with ``dA/dkappa_c`` assembled
from a unit coefficient field; plus central finite differences of ``J``.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import adjoint, compact, dense, plain


def _solve_dense(kappa, f):
    d = kappa.ndim
    A = dense.diffusion(kappa)
    u = np.zeros_like(f)
    inner = (slice(1, -1),) * d
    u[inner] = np.linalg.solve(A, f[inner].reshape(-1)).reshape(f[inner].shape)
    return u


@pytest.mark.parametrize("dim,L", [(2, 3), (3, 2)])
def test_gradient_matches_dense_brute_force(dim, L):
    n = 1 << L
    kappa = S.lognormal_kappa(dim, L, 0.3, 1)
    kobs = S.lognormal_kappa(dim, L, 0.3, 2)
    f = np.zeros((n + 1,) * dim)
    f[(slice(1, -1),) * dim] = 1.0
    u = _solve_dense(kappa, f)
    uobs = _solve_dense(kobs, f)
    lam = _solve_dense(kappa, adjoint.loss_grad_u(u, uobs))
    g = adjoint.grad_kappa(u, lam)
    ui, li = dense.interior(u), dense.interior(lam)
    for cell in np.ndindex(*kappa.shape):
        dA = dense.diffusion_derivative(kappa, cell)
        assert np.isclose(g[cell], -li @ dA @ ui, rtol=1e-10, atol=1e-14)


def test_gradient_matches_finite_differences():
    dim, L = 2, 3
    n = 1 << L
    kappa = S.lognormal_kappa(dim, L, 0.3, 3)
    f = S.smoothed_noise_rhs(dim, L, 7)
    uobs = _solve_dense(S.lognormal_kappa(dim, L, 0.3, 4), f)
    u = _solve_dense(kappa, f)
    lam = _solve_dense(kappa, adjoint.loss_grad_u(u, uobs))
    g = adjoint.grad_kappa(u, lam)
    rng = np.random.default_rng(0)
    for _ in range(3):
        delta = rng.standard_normal(kappa.shape)
        eps = 1e-6
        jp = adjoint.loss(_solve_dense(kappa * (1 + eps * delta), f), uobs)
        jm = adjoint.loss(_solve_dense(kappa * (1 - eps * delta), f), uobs)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * kappa * delta))
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_unit_kappa_diffusion_fmg_matches_poisson():
    dim, L = 3, 4
    n = 1 << L
    f = S.sine_rhs(dim, L)
    cfg_d = compact.Config(dim=dim, L=L, op="diffusion", vcycle_dtype=np.float64, quantize=False)
    cfg_p = compact.Config(dim=dim, L=L, vcycle_dtype=np.float64, quantize=False)
    ud, _ = compact.fmg_solve(f, cfg_d, np.ones((n,) * dim))
    up, _ = compact.fmg_solve(f, cfg_p)
    assert np.abs(ud - up).max() <= 1e-12 * np.abs(up).max()


def test_fmg_diffusion_converges_to_dense_solution():
    dim, L = 3, 3
    kappa = S.lognormal_kappa(dim, L, 0.3, 1)
    f = np.zeros(((1 << L) + 1,) * dim)
    f[(slice(1, -1),) * dim] = 1.0
    ud = _solve_dense(kappa, f)
    cfg = compact.Config(dim=dim, L=L, op="diffusion", vcycle_dtype=np.float64)
    uc = plain.vcycles_to_convergence(f, cfg, kappa)
    assert np.abs(uc - ud).max() <= 1e-12 * np.abs(ud).max()
