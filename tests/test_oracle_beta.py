"""Pins of the oracle's Eq. 3 operator (arbitrary neighbour coefficients):
beta = 1 reproduces the interior part of Fig. 3's system (and its boundary
columns), and beta = 4 eps_f / sum(eps_f) is the row-normalised conservative
operator, exactly."""

import numpy as np

from oracle import grid, inverse


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


def test_lu_inverse_with_a_row_exchange_is_exact():
    """A = [[1, -1, 0], [-1, 1, -1], [0, -1, 1]] (Eq. 3 with four inner
    coefficients of 4): natural-order elimination meets a zero second pivot, so
    only a pivoting LU inverts it; the inverse is the integer matrix
    -[[0, 1, 1], [1, 1, 1], [1, 1, 0]] (det A = -1), reached exactly."""
    beta = np.zeros((4, 3, 5))
    beta[3, 1, 1] = beta[2, 1, 2] = beta[3, 1, 2] = beta[2, 1, 3] = 4.0
    A, _ = grid.beta_operator(5, 3, beta)
    assert np.array_equal(A, np.array([[1.0, -1.0, 0.0], [-1.0, 1.0, -1.0], [0.0, -1.0, 1.0]]))
    assert np.array_equal(inverse.lu_inverse(A), -np.array([[0.0, 1.0, 1.0], [1.0, 1.0, 1.0], [1.0, 1.0, 0.0]]))


def test_lu_inverse_of_mixed_sign_coefficients_is_a_true_inverse():
    """beta ~ U(-3, 3): A X = I and X A = I to 1e-12 |A| |X| (max norms), the
    two-sided residual of an inverse."""
    g = np.random.default_rng(31)
    nx, ny = 17, 13
    A, _ = grid.beta_operator(nx, ny, g.uniform(-3.0, 3.0, (4, ny, nx)))
    X = inverse.lu_inverse(A)
    I = np.eye(A.shape[0])
    scale = np.max(np.abs(A)) * np.max(np.abs(X)) * A.shape[0] ** 0.5
    assert np.max(np.abs(A @ X - I)) <= 1e-12 * scale
    assert np.max(np.abs(X @ A - I)) <= 1e-12 * scale
