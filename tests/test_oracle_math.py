"""Pins of the oracle's operator and inverse to closed forms and invariants of
the 5-point discretisation (they hold exactly in exact arithmetic)."""

import numpy as np
import pytest

from oracle import apply, grid, inverse, metrics
from paper_1602_00001_amd import workloads


@pytest.mark.parametrize("nx,ny", [(5, 5), (12, 9), (20, 20), (7, 30)])
def test_lu_inverse_matches_dst_closed_form(nx, ny):
    """eps = 1: LU inverse of K equals the DST-I eigen-decomposition."""
    K, _ = grid.conservative_operator(nx, ny)
    G = inverse.lu_inverse(K)
    D = inverse.dst_inverse(nx, ny)
    assert np.linalg.norm(G - D) / np.linalg.norm(D) < 1e-12
    rho = np.random.default_rng(0).uniform(-1, 1, (G.shape[0], 3))
    assert np.max(metrics.rel_l2_per_rhs(G @ rho, D @ rho)) < 1e-12


def test_dst_rows_match_full():
    D = inverse.dst_inverse(17, 11)
    rows = [0, 4, 44, D.shape[0] - 1]
    assert np.allclose(inverse.dst_inverse_rows(17, 11, rows), D[rows], rtol=0, atol=1e-15)


def test_dst_inverse_is_inverse():
    """K @ dst_inverse = I (independent of LU)."""
    K, _ = grid.conservative_operator(14, 10)
    D = inverse.dst_inverse(14, 10)
    assert np.max(np.abs(K @ D - np.eye(K.shape[0]))) < 1e-13


@pytest.mark.parametrize("n", [32, 64])
def test_sin_sin_is_exact_discrete_eigenvector(n):
    """u = sin(pi x) sin(pi y): Laplacian u = -2 pi^2 u.  The 5-point solution is
    c(h) * u at the nodes, c(h) = (pi h / 2)^2 / sin^2(pi h / 2)."""
    X, Y, h = workloads.coords(n)
    ue = np.sin(np.pi * X) * np.sin(np.pi * Y)
    rho = workloads.interior(-2 * np.pi ** 2 * ue)
    G = inverse.dst_inverse(n, n) if n > 40 else inverse.lu_inverse(grid.conservative_operator(n, n)[0])
    u = apply.plain_apply(G, rho[:, None], h)[:, 0]
    c = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    assert np.max(np.abs(u - c * workloads.interior(ue))) < 1e-12
    # Eq. 6 error of the discrete solution is c(h) - 1
    assert abs(metrics.eq6_error(u, workloads.interior(ue)) - (c - 1)) < 1e-10 * c


def test_second_order_convergence():
    """Error against sin(pi x) sin(pi y) falls by ~4x when h halves."""
    errs = []
    for n in (17, 33, 65):
        X, Y, h = workloads.coords(n)
        ue = np.sin(np.pi * X) * np.sin(np.pi * Y)
        rho = workloads.interior(-2 * np.pi ** 2 * ue)
        u = apply.plain_apply(inverse.dst_inverse(n, n), rho[:, None], h)[:, 0]
        errs.append(metrics.eq6_error(u, workloads.interior(ue)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.95 < r2 < 4.05


@pytest.mark.parametrize("seed", [0, 1])
def test_constant_dirichlet_data_gives_constant_solution(seed):
    """Any eps: u_B = 1 and rho = 0 give u = 1 (rows of K sum to the boundary faces)."""
    g = np.random.default_rng(seed)
    nx, ny = 13, 9
    eps = workloads.random_eps(nx, ny, g)
    ub = np.ones((ny, nx))
    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    G = inverse.lu_inverse(K)
    w = apply.lift(G, bB)
    u = apply.plain_apply(G, np.zeros((K.shape[0], 1)), 0.1, w)
    assert np.max(np.abs(u - 1.0)) < 1e-13


def test_bilinear_data_reproduced_exactly():
    """eps = 1: a + b x + c y + d xy is discrete-harmonic; with rho = 0 and that
    boundary data the interior solution equals it at the nodes."""
    n = 15
    X, Y, h = workloads.coords(n)
    ue = 0.3 + 1.7 * X - 0.6 * Y + 2.2 * X * Y
    K, bB = grid.conservative_operator(n, n, None, ue)
    u = apply.plain_apply(inverse.lu_inverse(K), np.zeros((K.shape[0], 1)), h, apply.lift(inverse.lu_inverse(K), bB))
    assert np.max(np.abs(u[:, 0] - workloads.interior(ue))) < 1e-13


def test_variable_eps_operator_matches_flux_form():
    """K u equals the flux sum computed face by face from nodal values."""
    g = np.random.default_rng(3)
    nx, ny = 8, 6
    eps = workloads.random_eps(nx, ny, g)
    ub = g.standard_normal((ny, nx))
    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    u_int = g.standard_normal(K.shape[0])
    U = grid.interior_to_nodes(nx, ny, u_int, ub)
    flux = np.zeros((ny, nx))
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            for (k, l) in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)):
                flux[i, j] += 0.5 * (eps[i, j] + eps[k, l]) * (U[i, j] - U[k, l])
    assert np.allclose(K @ u_int - bB, grid.nodes_to_interior(nx, ny, flux), atol=1e-13)


@pytest.mark.parametrize("kind", ["sincos", "lognormal", "uniform"])
def test_inverse_invariants(kind):
    """G = K^{-1} is symmetric, entrywise positive, with each row's maximum on
    the diagonal (discrete maximum principle), and constants are preserved."""
    n = 20
    g = np.random.default_rng(11)
    eps = {"sincos": workloads.eps_sincos(n), "lognormal": workloads.eps_lognormal(n, g),
           "uniform": workloads.random_eps(n, n, g)}[kind]
    K, _ = grid.conservative_operator(n, n, eps)
    G = inverse.lu_inverse(K)
    assert np.max(np.abs(G - G.T)) < 1e-14 * np.max(np.abs(G))
    assert np.min(G) > 0
    assert np.all(np.argmax(G, axis=1) == np.arange(G.shape[0]))


def test_nonpositive_eps_breaks_spd():
    """eps with a negative region gives a K that is not positive definite."""
    n = 10
    eps = np.ones((n, n))
    eps[3:7, 3:7] = -2.0
    K, _ = grid.conservative_operator(n, n, eps)
    assert np.min(np.linalg.eigvalsh(K)) < 0


def test_banded_operator_matches_dense():
    g = np.random.default_rng(5)
    nx, ny = 9, 7
    eps = workloads.random_eps(nx, ny, g)
    K, _ = grid.conservative_operator(nx, ny, eps)
    ab = grid.conservative_operator_banded(nx, ny, eps)
    N, bw = K.shape[0], ab.shape[0] - 1
    for d in range(bw + 1):
        assert np.array_equal(ab[d, :N - d], np.diag(K, -d))
    assert np.all(np.abs(np.tril(K, -bw - 1)) == 0)
