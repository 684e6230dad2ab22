"""Pins of the oracle's derivatives: adjoint identity, eps-gradient against
central finite differences of freshly re-solved systems, and the banded solve
against the dense inverse."""

import numpy as np
import pytest

from oracle import apply, grad, grid, inverse, quant
from paper_1602_00001_amd import workloads


def test_adjoint_dot_product_identity_quantised():
    """<G^ x, y> = <x, G^T y> exactly on the integer parts."""
    g = np.random.default_rng(2)
    N = 25
    G = g.standard_normal((N, N))
    qG, e = quant.quantize_rows(G, 2)
    x = g.integers(-1000, 1000, (N, 3))
    y = g.integers(-1000, 1000, (N, 3))
    lhs = np.sum((qG @ x) * y, axis=0)
    rhs = np.sum(x * (qG.T @ y), axis=0)
    assert np.array_equal(lhs, rhs)


def test_banded_solve_matches_dense():
    g = np.random.default_rng(3)
    nx, ny, h = 11, 9, 0.1
    eps = workloads.random_eps(nx, ny, g)
    ub = g.standard_normal((ny, nx))
    rho = g.standard_normal(((nx - 2) * (ny - 2), 2))
    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    G = inverse.lu_inverse(K)
    u_dense = apply.plain_apply(G, rho, h, apply.lift(G, bB))
    u_band = grad.banded_solve(nx, ny, h, eps, rho, ub)
    assert np.max(np.abs(u_dense - u_band)) < 1e-12 * np.max(np.abs(u_dense))


@pytest.mark.parametrize("with_boundary", [False, True])
def test_grad_eps_matches_central_differences(with_boundary):
    """dLoss/deps from (u, lambda) equals central differences of the re-solved
    loss along random directions, to 1e-6 relative."""
    g = np.random.default_rng(4 + with_boundary)
    nx, ny = 12, 10
    h = 1.0 / (nx - 1)
    N = (nx - 2) * (ny - 2)
    eps = 1.0 + 0.5 * g.uniform(0, 1, (ny, nx))
    ub = g.standard_normal((ny, nx)) if with_boundary else None
    rho = g.standard_normal((N, 3))
    sample = np.sort(g.choice(N, 15, replace=False))
    d = g.standard_normal((15, 3)) * 0.01

    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    G = inverse.lu_inverse(K)
    u = apply.plain_apply(G, rho, h, apply.lift(G, bB))
    gu = grad.sampling_loss_grad_u(u, sample, d)
    lam = grad.adjoint(G, gu, h)
    ge = grad.grad_eps_nodes(nx, ny, h, u, lam, ub)

    def loss(e):
        return grad.sampling_loss(nx, ny, h, e, rho, sample, d, ub)

    for t in range(3):
        v = g.standard_normal((ny, nx))
        fd = grad.central_difference(loss, eps, v, 1e-6)
        an = float(np.sum(ge * v))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-30), (fd, an)

    # dLoss/drho = lambda, also against central differences
    for t in range(2):
        v = g.standard_normal(rho.shape)
        fd = grad.central_difference(lambda r: grad.sampling_loss(nx, ny, h, eps, r, sample, d, ub), rho, v, 1e-6)
        an = float(np.sum(lam * v))
        assert abs(fd - an) <= 1e-6 * abs(fd)


def test_grad_eps_faces_between_boundary_nodes_do_not_count():
    """eps at a corner node touches only boundary-boundary faces: zero gradient."""
    g = np.random.default_rng(8)
    nx, ny, h = 7, 6, 0.2
    N = (nx - 2) * (ny - 2)
    u = g.standard_normal((N, 2))
    lam = g.standard_normal((N, 2))
    ge = grad.grad_eps_nodes(nx, ny, h, u, lam, g.standard_normal((ny, nx)))
    for (i, j) in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        assert ge[i, j] == 0.0


def test_cancellation_free_central_difference_matches_plain_form():
    """The term-by-term central difference equals [L(+) - L(-)]/(2 delta) (the
    same number up to the rounding of the plain form) along eps and rho."""
    g = np.random.default_rng(13)
    nx, ny = 11, 9
    h = 1.0 / (nx - 1)
    N = (nx - 2) * (ny - 2)
    eps = 1.0 + g.uniform(0, 1, (ny, nx))
    rho = g.standard_normal((N, 2))
    sample = np.sort(g.choice(N, 12, replace=False))
    d = 0.01 * g.standard_normal((12, 2))
    v = g.standard_normal((ny, nx))
    a = grad.sampling_loss_central_difference(nx, ny, h, eps, rho, sample, d, v_eps=v, delta=1e-4)
    b = grad.central_difference(lambda e: grad.sampling_loss(nx, ny, h, e, rho, sample, d), eps, v, 1e-4)
    assert abs(a - b) <= 1e-9 * abs(b)
    w = g.standard_normal(rho.shape)
    a = grad.sampling_loss_central_difference(nx, ny, h, eps, rho, sample, d, v_rho=w, delta=1e-4)
    b = grad.central_difference(lambda r: grad.sampling_loss(nx, ny, h, eps, r, sample, d), rho, w, 1e-4)
    assert abs(a - b) <= 1e-9 * abs(b)


def test_extended_operator_matches_dense_K():
    g = np.random.default_rng(14)
    nx, ny = 10, 8
    eps = workloads.random_eps(nx, ny, g)
    K, _ = grid.conservative_operator(nx, ny, eps)
    u = g.standard_normal((K.shape[0], 3))
    assert np.allclose(grad.apply_operator_extended(nx, ny, eps, u).astype(np.float64), K @ u, rtol=0, atol=1e-13)


def test_refined_banded_solve_is_more_accurate():
    """Against an exact rational-free reference: the dense solve refined with the
    same extended residual, and the residual norms before and after."""
    g = np.random.default_rng(15)
    nx, ny = 41, 37
    h = 1.0 / (nx - 1)
    eps = 1.0 + 0.5 * g.uniform(0, 1, (ny, nx))
    ub = g.standard_normal((ny, nx))
    rho = g.standard_normal(((nx - 2) * (ny - 2), 2))
    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    u_plain = grad.banded_solve(nx, ny, h, eps, rho, ub)
    u_ref = grad.banded_solve_refined(nx, ny, h, eps, rho, ub)
    rhs = (-(h * h)) * rho.astype(np.longdouble) + bB.astype(np.longdouble)[:, None]
    res_plain = np.abs(rhs - grad.apply_operator_extended(nx, ny, eps, u_plain)).max()
    res_ref = np.abs(rhs - grad.apply_operator_extended(nx, ny, eps, u_ref)).max()
    assert res_ref <= res_plain
    assert np.max(np.abs(u_ref - u_plain)) <= 1e-12 * np.max(np.abs(u_plain))


def test_grad_eps_3d_matches_central_differences():
    """3-D face rule against central differences of the dense re-solved loss."""
    g = np.random.default_rng(61)
    nx, ny, nz = 7, 6, 5
    h = 1.0 / (nx - 1)
    eps = 1.0 + 0.5 * g.uniform(0, 1, (nz, ny, nx))
    ub = g.standard_normal((nz, ny, nx))
    N = (nx - 2) * (ny - 2) * (nz - 2)
    rho = g.standard_normal((N, 2))
    sample = np.sort(g.choice(N, 10, replace=False))
    d = 0.01 * g.standard_normal((10, 2))

    def solve(e):
        K, bB = grid.conservative_operator_3d(nx, ny, nz, e, ub)
        return np.linalg.solve(K, -(h * h) * rho + bB[:, None]), K

    def loss(e):
        u, _ = solve(e)
        r = u[sample] - d
        return float(np.sum(r * r))

    u, K = solve(eps)
    gu = grad.sampling_loss_grad_u(u, sample, d)
    lam = grad.adjoint(np.linalg.inv(K), gu, h)
    ge = grad.grad_eps_nodes_3d(nx, ny, nz, h, u, lam, ub)
    for t in range(3):
        v = g.standard_normal((nz, ny, nx))
        fd = grad.central_difference(loss, eps, v, 1e-6)
        an = float(np.sum(ge * v))
        assert abs(fd - an) <= 1e-6 * abs(fd), (fd, an)


def test_grad_eps_general_matches_central_differences():
    """Per-direction gradients on a non-uniform grid against central differences
    of the dense re-solved loss, perturbing eps_x and eps_y separately; on a
    uniform grid with one field their sum is the uniform nodal gradient."""
    g = np.random.default_rng(67)
    nx, ny = 8, 7
    x = np.concatenate([[0.0], np.sort(g.uniform(0.05, 0.95, nx - 2)), [1.0]])
    y = np.concatenate([[0.0], np.sort(g.uniform(0.05, 0.95, ny - 2)), [1.0]])
    ex = g.uniform(0.5, 2.0, (ny, nx))
    ey = g.uniform(0.5, 2.0, (ny, nx))
    ub = g.standard_normal((ny, nx))
    N = (nx - 2) * (ny - 2)
    rho = g.standard_normal((N, 3))
    sample = np.sort(g.choice(N, 9, replace=False))
    d = 0.01 * g.standard_normal((9, 3))

    def solve(a, b):
        K, bB, A = grid.conservative_operator_general(x, y, a, b, ub)
        return np.linalg.solve(K, -A[:, None] * rho + bB[:, None]), K, A

    def loss(a, b):
        u, _, _ = solve(a, b)
        r = u[sample] - d
        return float(np.sum(r * r))

    u, K, A = solve(ex, ey)
    gu = grad.sampling_loss_grad_u(u, sample, d)
    Gp = np.linalg.inv(K) * A[None, :]                 # the stored inverse K^{-1} diag(A)
    lam = -(Gp.T @ gu)
    gx, gy = grad.grad_eps_general(x, y, u, lam, ub)
    for t in range(2):
        v = g.standard_normal((ny, nx))
        fdx = grad.central_difference(lambda e: loss(e, ey), ex, v, 1e-6)
        fdy = grad.central_difference(lambda e: loss(ex, e), ey, v, 1e-6)
        assert abs(fdx - float(np.sum(gx * v))) <= 1e-6 * abs(fdx), (fdx, float(np.sum(gx * v)))
        assert abs(fdy - float(np.sum(gy * v))) <= 1e-6 * abs(fdy), (fdy, float(np.sum(gy * v)))

    # uniform grid, one field: gx + gy is the uniform gradient (lambda carries A = h^2)
    n = 7
    h = 1.0 / (n - 1)
    t = np.arange(n) * h
    eps = g.uniform(0.5, 2.0, (n, n))
    Nn = (n - 2) ** 2
    uu = g.standard_normal((Nn, 2))
    ll = g.standard_normal((Nn, 2))
    gx, gy = grad.grad_eps_general(t, t, uu, ll, None)
    ref = grad.grad_eps_nodes(n, n, h, uu, ll, None)
    assert np.allclose(gx + gy, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_grad_beta_matches_central_differences():
    """Eq. 3 with arbitrary coefficients: dLoss/dbeta against central
    differences of the dense re-solved loss (the adjoint output is A^{-T} g)."""
    g = np.random.default_rng(71)
    nx, ny = 8, 7
    beta = g.uniform(0.2, 1.0, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    N = (nx - 2) * (ny - 2)
    rho = g.standard_normal((N, 2))
    sample = np.sort(g.choice(N, 9, replace=False))
    d = 0.01 * g.standard_normal((9, 2))

    def solve(b):
        A, bB = grid.beta_operator(nx, ny, b, ub)
        return np.linalg.solve(A, rho + bB[:, None]), A

    def loss(b):
        u, _ = solve(b)
        r = u[sample] - d
        return float(np.sum(r * r))

    u, A = solve(beta)
    gu = grad.sampling_loss_grad_u(u, sample, d)
    lam = np.linalg.solve(A.T, gu)
    gb = grad.grad_beta(nx, ny, u, lam, ub)
    assert np.all(gb[:, 0, :] == 0) and np.all(gb[:, :, -1] == 0)
    for _ in range(3):
        v = g.standard_normal((4, ny, nx))
        fd = grad.central_difference(loss, beta, v, 1e-6)
        an = float(np.sum(gb * v))
        assert abs(fd - an) <= 1e-6 * abs(fd), (fd, an)
