"""Pins of the oracle's 3-D (7-point) operator and inverse: an independent
Kronecker construction, the closed-form (DST) inverse, exact reproduction of
constant Dirichlet data, the discrete eigenvector sin(pi x) sin(pi y) sin(pi z),
and the M-matrix invariants."""

import numpy as np

from oracle import apply, grid, inverse


def _tri(m):
    return 2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)


def test_eps_one_equals_kronecker_form():
    nx, ny, nz = 7, 6, 5
    K, bB = grid.conservative_operator_3d(nx, ny, nz)
    mx, my, mz = nx - 2, ny - 2, nz - 2
    Iz, Iy, Ix = np.eye(mz), np.eye(my), np.eye(mx)
    ref = (np.kron(_tri(mz), np.kron(Iy, Ix)) + np.kron(Iz, np.kron(_tri(my), Ix))
           + np.kron(Iz, np.kron(Iy, _tri(mx))))
    assert np.array_equal(K, ref)
    assert not bB.any()


def test_dst_inverse_3d_inverts_the_operator():
    nx, ny, nz = 8, 7, 6
    K, _ = grid.conservative_operator_3d(nx, ny, nz)
    D = inverse.dst_inverse_3d(nx, ny, nz)
    assert np.max(np.abs(K @ D - np.eye(K.shape[0]))) < 1e-12
    L = inverse.lu_inverse(K)
    assert np.max(np.abs(L - D)) < 1e-12 * np.max(np.abs(D))


def test_constant_dirichlet_data_is_reproduced():
    """u_B = 1 on the boundary, rho = 0: the solution is 1 everywhere, for any eps."""
    g = np.random.default_rng(31)
    nx, ny, nz = 7, 8, 6
    eps = g.uniform(0.5, 2.0, (nz, ny, nx))
    K, bB = grid.conservative_operator_3d(nx, ny, nz, eps, np.ones((nz, ny, nx)))
    G = inverse.lu_inverse(K)
    assert np.max(np.abs(G @ bB - 1.0)) < 1e-13
    assert np.allclose(K, K.T, rtol=0, atol=0)
    assert np.all(G > 0)
    assert np.all(np.argmax(G, axis=1) == np.arange(G.shape[0]))


def test_sin_sin_sin_is_a_discrete_eigenvector():
    """For Delta u = rho with rho = -3 pi^2 sin(pi x) sin(pi y) sin(pi z) and zero
    Dirichlet data, the 7-point solution is c(h) times the exact one at the nodes,
    c(h) = (pi h / 2)^2 / sin^2(pi h / 2)."""
    n = 9
    h = 1.0 / (n - 1)
    t = np.arange(1, n - 1) * h
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    u_exact = (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)).reshape(-1)
    rho = -3.0 * np.pi ** 2 * u_exact
    G = inverse.dst_inverse_3d(n, n, n)
    u = apply.plain_apply(G, rho[:, None], h, None)[:, 0]
    c = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    assert np.max(np.abs(u - c * u_exact)) < 1e-10 * np.max(np.abs(u_exact))
