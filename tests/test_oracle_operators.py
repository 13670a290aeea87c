"""Pins of the oracle's operators, transfers and smoothers (no GPU).

Each check compares the vectorised oracle against something written
independently: dense Kronecker assemblies, closed-form eigenpairs of the
discrete Laplacian, hat functions for interpolation, and an explicitly
ordered dense Gauss-Seidel.
"""
import itertools

import numpy as np
import pytest

from oracle import dense, grid


def _rand_level(dim, level, seed):
    n = 1 << level
    u = np.zeros((n,) * dim)
    u[(slice(1, None),) * dim] = np.random.default_rng(seed).standard_normal((n - 1,) * dim)
    return u


def _apply_dense_columns(lv):
    d, n = lv.dim, lv.n
    m = (n - 1) ** d
    A = np.zeros((m, m))
    for j in range(m):
        e = np.zeros((n,) * d)
        e_in = np.zeros((n - 1,) * d)
        e_in.flat[j] = 1.0
        e[(slice(1, None),) * d] = e_in
        A[:, j] = lv.apply(e, np.float64)[(slice(1, None),) * d].reshape(-1)
    return A


@pytest.mark.parametrize("dim,level", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_poisson_matches_kronecker_sum(dim, level):
    A = _apply_dense_columns(grid.Level(dim, level))
    K = dense.poisson(dim, level)
    assert np.array_equal(A, K)
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("dim,level,k", [(2, 5, (1, 1)), (2, 5, (3, 7)), (3, 4, (1, 2, 5))])
def test_sine_mode_is_eigenvector(dim, level, k):
    # s = prod_a sin(k_a pi x_a) has eigenvalue sum_a 4 h**-2 sin(k_a pi h / 2)**2
    n = 1 << level
    h = 1.0 / n
    x = np.arange(n) * h
    s = np.ones((n,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        s = s * np.sin(k[ax] * np.pi * x).reshape(shape)
    lam = sum(4.0 / h ** 2 * np.sin(kk * np.pi * h / 2) ** 2 for kk in k)
    As = grid.Level(dim, level).apply(s, np.float64)
    inner = (slice(1, None),) * dim
    assert np.allclose(As[inner], lam * s[inner], rtol=1e-12, atol=1e-12 * lam)


@pytest.mark.parametrize("dim,level", [(2, 3), (3, 2)])
def test_diffusion_matches_edge_assembly(dim, level):
    n = 1 << level
    kappa = np.exp(np.random.default_rng(7).standard_normal((n,) * dim))
    lv = grid.Level(dim, level, "diffusion", kappa)
    A = _apply_dense_columns(lv)
    K = dense.diffusion(kappa)
    assert np.allclose(A, K, rtol=1e-13, atol=0)
    assert np.allclose(A, A.T, rtol=1e-13)
    assert np.allclose(np.diag(K), lv.diag(np.float64).reshape(-1), rtol=1e-14)


@pytest.mark.parametrize("dim,level", [(2, 4), (3, 3)])
def test_diffusion_with_unit_kappa_is_poisson(dim, level):
    n = 1 << level
    u = _rand_level(dim, level, 3)
    a = grid.Level(dim, level, "diffusion", np.ones((n,) * dim)).apply(u, np.float64)
    b = grid.Level(dim, level).apply(u, np.float64)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-11 * np.abs(b).max())


@pytest.mark.parametrize("dim,level", [(2, 3), (2, 5), (3, 3)])
def test_prolongation_matches_kronecker(dim, level):
    m = 1 << (level - 1)
    c = _rand_level(dim, level - 1, 11)
    fine = grid.prolong(c, np.float64)
    P = dense.prolongation(dim, level)
    ref = P @ c[(slice(1, None),) * dim].reshape(-1)
    assert np.allclose(fine[(slice(1, None),) * dim].reshape(-1), ref, rtol=1e-15, atol=1e-15)
    # boundary nodes stay zero
    for ax in range(dim):
        sl = [slice(None)] * dim
        sl[ax] = 0
        assert not np.any(fine[tuple(sl)])
    assert fine.shape == ((2 * m,) * dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_of_hat_function(dim):
    level = 4
    n = 1 << level
    m = n // 2
    J = (3,) * dim if dim == 2 else (2, 5, 3)
    c = np.zeros((m,) * dim)
    c[J] = 1.0
    fine = grid.prolong(c, np.float64)
    H = 1.0 / m
    xs = np.arange(n) / n
    expect = np.ones((n,) * dim)
    for ax in range(dim):
        hat = np.maximum(0.0, 1.0 - np.abs(xs - J[ax] * H) / H)
        shape = [1] * dim
        shape[ax] = n
        expect = expect * hat.reshape(shape)
    assert np.array_equal(fine, expect)


@pytest.mark.parametrize("dim,level", [(2, 3), (2, 5), (3, 3)])
def test_restriction_is_scaled_transpose(dim, level):
    f = _rand_level(dim, level, 13)
    coarse = grid.restrict(f, np.float64)
    P = dense.prolongation(dim, level)
    ref = (0.5 ** dim) * P.T @ f[(slice(1, None),) * dim].reshape(-1)
    assert np.allclose(coarse[(slice(1, None),) * dim].reshape(-1), ref, rtol=1e-14, atol=1e-15)


def test_full_weighting_of_constant():
    f = np.zeros((16, 16, 16))
    f[1:, 1:, 1:] = 1.0
    c = grid.restrict(f, np.float64)
    assert np.all(c[2:-1, 2:-1, 2:-1] == 1.0)


@pytest.mark.parametrize("dim,omega", [(2, 0.8), (3, 6.0 / 7.0)])
def test_jacobi_multiplier_on_sine_mode(dim, omega):
    level = 4
    n = 1 << level
    h = 1.0 / n
    k = (3, 5, 2)[:dim]
    x = np.arange(n) * h
    s = np.ones((n,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        s = s * np.sin(k[ax] * np.pi * x).reshape(shape)
    lv = grid.Level(dim, level)
    y = grid.smooth(lv, s, np.zeros_like(s), 1, "wjacobi", omega, np.float64)
    mult = 1.0 - omega * (1.0 - np.mean([np.cos(kk * np.pi * h) for kk in k]))
    inner = (slice(1, None),) * dim
    assert np.allclose(y[inner], mult * s[inner], atol=1e-13)


@pytest.mark.parametrize("dim,level,op", [(2, 3, "poisson"), (3, 2, "poisson"), (3, 2, "diffusion")])
def test_rbgs_equals_ordered_dense_gauss_seidel(dim, level, op):
    n = 1 << level
    kappa = np.exp(np.random.default_rng(1).standard_normal((n,) * dim)) if op == "diffusion" else None
    lv = grid.Level(dim, level, op, kappa)
    A = dense.poisson(dim, level) if op == "poisson" else dense.diffusion(kappa)
    rhs = _rand_level(dim, level, 5)
    y0 = _rand_level(dim, level, 6)
    inner = (slice(1, None),) * dim
    nodes = list(itertools.product(range(1, n), repeat=dim))
    red = [i for i, p in enumerate(nodes) if sum(p) % 2 == 0]
    black = [i for i, p in enumerate(nodes) if sum(p) % 2 == 1]
    order = red + black
    Ap = A[np.ix_(order, order)]
    b = rhs[inner].reshape(-1)[order]
    y = y0[inner].reshape(-1)[order]
    DL = np.tril(Ap)
    U = Ap - DL
    for _ in range(2):
        y = np.linalg.solve(DL, b - U @ y)
    got = grid.smooth(lv, y0, rhs, 2, "rbgs", 1.0, np.float64)[inner].reshape(-1)[order]
    assert np.allclose(got, y, rtol=1e-12, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("dim,op", [(2, "poisson"), (3, "poisson"), (3, "diffusion")])
def test_coarse_solve_level_two(dim, op):
    kappa = np.exp(np.random.default_rng(2).standard_normal((4,) * dim)) if op == "diffusion" else None
    lv = grid.Level(dim, 2, op, kappa)
    g = _rand_level(dim, 2, 9)
    y = grid.coarse_solve(lv, g)
    A = dense.poisson(dim, 2) if op == "poisson" else dense.diffusion(kappa)
    inner = (slice(1, None),) * dim
    ref = np.linalg.solve(A, g[inner].reshape(-1))
    assert np.allclose(y[inner].reshape(-1), ref, rtol=1e-13)


def test_coarse_solve_single_node():
    for dim in (2, 3):
        lv = grid.Level(dim, 1)
        g = np.zeros((2,) * dim)
        g[(1,) * dim] = 3.0
        y = grid.coarse_solve(lv, g)
        assert y[(1,) * dim] == 3.0 / (2 * dim * 4.0)


def test_kappa_coarsening_mean():
    k = np.arange(64, dtype=float).reshape(4, 4, 4)
    c = grid.coarsen_kappa(k)
    assert c.shape == (2, 2, 2)
    assert c[1, 0, 1] == np.mean(k[2:4, 0:2, 2:4])


def test_ldlt_solve_hand_case_and_library():
    # hand case: A = [[4, 2], [2, 3]]: d = (4, 2), l_10 = 1/2; b = (2, 1)
    # gives z = (2, 0), x = (1/2, 0), exactly
    x = grid.ldlt_solve(np.array([[4.0, 2.0], [2.0, 3.0]]), np.array([2.0, 1.0]))
    assert x[0] == 0.5 and x[1] == 0.0
    rng = np.random.default_rng(3)
    for m in (1, 5, 27):
        M = rng.standard_normal((m, m))
        A = M @ M.T + m * np.eye(m)
        b = rng.standard_normal(m)
        ref = np.linalg.solve(A, b)
        assert np.allclose(grid.ldlt_solve(A, b), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
