"""Pins of the oracle's non-uniform, per-direction-permittivity operator: the
uniform special case, exact bilinear data on a non-uniform grid, constant
Dirichlet data for anisotropic eps, the closed-form inverse for constant
anisotropic eps, and second-order convergence on a stretched grid."""

import numpy as np

from oracle import grid, inverse


def _stretched(n, a):
    """Smoothly stretched nodes on [0, 1]: x = t + a sin(2 pi t) / (2 pi)."""
    t = np.linspace(0.0, 1.0, n)
    return t + a * np.sin(2 * np.pi * t) / (2 * np.pi)


def test_uniform_case_reduces_to_the_standard_operator():
    nx, ny = 9, 17                      # power-of-two spacing: every face weight is exact
    h = 0.125
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    g = np.random.default_rng(41)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    ub = g.standard_normal((ny, nx))
    K, bB, A = grid.conservative_operator_general(x, y, eps, eps, ub)
    K0, b0 = grid.conservative_operator(nx, ny, eps, ub)
    assert np.array_equal(K, K0) and np.array_equal(bB, b0)
    assert np.all(A == h * h)


def test_bilinear_data_exact_on_a_nonuniform_grid():
    x = _stretched(11, 0.6)
    y = _stretched(9, -0.4)
    X, Y = np.meshgrid(x, y)
    u = 0.3 + 1.2 * X - 0.7 * Y + 2.1 * X * Y
    K, bB, A = grid.conservative_operator_general(x, y, None, None, u)
    sol = np.linalg.solve(K, bB)
    assert np.max(np.abs(sol - u[1:-1, 1:-1].reshape(-1))) < 1e-12


def test_constant_dirichlet_data_anisotropic():
    g = np.random.default_rng(42)
    x = np.sort(np.concatenate([[0.0, 1.0], g.uniform(0, 1, 9)]))
    y = np.sort(np.concatenate([[0.0, 1.0], g.uniform(0, 1, 7)]))
    ex = g.uniform(0.2, 3.0, (y.size, x.size))
    ey = g.uniform(0.2, 3.0, (y.size, x.size))
    K, bB, _ = grid.conservative_operator_general(x, y, ex, ey, np.ones((y.size, x.size)))
    assert np.max(np.abs(np.linalg.solve(K, bB) - 1.0)) < 1e-12
    assert np.array_equal(K, K.T)
    G = inverse.lu_inverse(K)
    assert np.all(G > 0)


def test_constant_anisotropic_eps_closed_form():
    """eps_x = a, eps_y = b on a uniform grid: K = b T_y (x) I + a I (x) T_x, whose
    inverse is diagonal in the DST basis with eigenvalues b ly + a lx."""
    nx, ny, a, b = 10, 8, 2.5, 0.75
    h = 1.0 / 8.0
    K, _, _ = grid.conservative_operator_general(np.arange(nx) * h, np.arange(ny) * h,
                                                 np.full((ny, nx), a), np.full((ny, nx), b))
    Sy, ly = inverse.dst_basis(ny - 2)
    Sx, lx = inverse.dst_basis(nx - 2)
    V = np.kron(Sy, Sx)
    lam = (b * ly[:, None] + a * lx[None, :]).reshape(-1)
    D = (V / lam[None, :]) @ V.T
    assert np.max(np.abs(K @ D - np.eye(K.shape[0]))) < 1e-12


def test_second_order_on_a_stretched_grid():
    """u = sin(pi x) sin(pi y), Delta u = -2 pi^2 u, zero Dirichlet data: the max
    error falls by about 4 when the stretched grid is refined by 2."""
    errs = []
    for n in (17, 33):
        x = _stretched(n, 0.5)
        y = _stretched(n, 0.5)
        K, bB, A = grid.conservative_operator_general(x, y)
        X, Y = np.meshgrid(x[1:-1], y[1:-1])
        ue = (np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
        rho = -2 * np.pi ** 2 * ue
        u = np.linalg.solve(K, -A * rho + bB)
        errs.append(np.max(np.abs(u - ue)))
    assert 3.3 < errs[0] / errs[1] < 4.7, errs
