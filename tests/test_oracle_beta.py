"""Pins of the oracle's Eq. 3 operator (arbitrary neighbour coefficients):
beta = 1 reproduces the interior part of Fig. 3's system (and its boundary
columns), and beta = 4 eps_f / sum(eps_f) is the row-normalised conservative
operator, exactly."""

import numpy as np

from oracle import grid


def test_beta_one_is_the_interior_of_fig3():
    nx, ny = 7, 6
    g = np.random.default_rng(51)
    ub = g.standard_normal((ny, nx))
    A, bB = grid.beta_operator(nx, ny, np.ones((4, ny, nx)), ub)
    full = grid.paper_full_matrix(nx, ny)
    inner = [i * nx + j for i in range(1, ny - 1) for j in range(1, nx - 1)]
    outer = [i * nx + j for i in range(ny) for j in range(nx) if grid.is_boundary(nx, ny, i, j)]
    assert np.array_equal(A, full[np.ix_(inner, inner)])
    assert np.allclose(bB, -full[np.ix_(inner, outer)] @ ub.reshape(-1)[outer], rtol=0, atol=1e-15)


def test_row_normalised_conservative_operator():
    nx, ny = 8, 7
    g = np.random.default_rng(52)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    K, _ = grid.conservative_operator(nx, ny, eps)
    beta = np.zeros((4, ny, nx))
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            faces = [grid.face_eps(eps, i, j, i + di, j + dj) for (di, dj) in grid.BETA_DIRECTIONS]
            total = sum(faces)
            for d, ef in enumerate(faces):
                beta[d, i, j] = 4.0 * ef / total
    A, _ = grid.beta_operator(nx, ny, beta)
    assert np.array_equal(A, K / np.diag(K)[:, None])


def test_m_matrix_invariants_without_symmetry():
    """For the paper's coefficients (beta_d = 4 eps_f / sum of the node's face
    eps) A = D^{-1} K with D = diag(K): A is not symmetric, but it is an
    M-matrix, so A^{-1} is entrywise positive (connected grid), A^{-1} D^{-1} =
    K^{-1} is symmetric, and constant Dirichlet data give the constant solution."""
    from oracle import inverse
    nx, ny = 9, 8
    g = np.random.default_rng(53)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    beta = np.zeros((4, ny, nx))
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            faces = [grid.face_eps(eps, i, j, i + di, j + dj) for (di, dj) in grid.BETA_DIRECTIONS]
            beta[:, i, j] = 4.0 * np.array(faces) / sum(faces)
    A, bB = grid.beta_operator(nx, ny, beta, np.ones((ny, nx)))
    Ainv = inverse.lu_inverse(A)
    assert np.max(np.abs(A - A.T)) > 1e-3
    assert np.all(Ainv > 0)
    K, _ = grid.conservative_operator(nx, ny, eps)
    S = Ainv / np.diag(K)[None, :]
    assert np.max(np.abs(S - S.T)) <= 1e-13 * np.max(np.abs(S))
    assert np.allclose(Ainv @ bB, 1.0, rtol=0, atol=1e-13)
