"""Eq. 3 with arbitrary (non-symmetric) neighbour coefficients: the inverse
computed on the host ("any standard matrix inversion method") and imported,
and the GPU LU build; the apply and the adjoint run the same GPU kernels.  The adjoint must be
the true transpose: FP64 against the oracle's -G^T g, int8 bit for bit against
the oracle's integer product with the transposed digit planes."""

import numpy as np
import pytest

from oracle import apply, grad, grid, inverse, metrics, quant
from tests.gpu_util import announce, dev, host, oracle_int8, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("nx,ny", [(12, 9), (40, 31)])
def test_beta_operator_apply_and_adjoint(torch, nx, ny):
    from paper_1602_00001_amd import pinv
    announce(f"Eq. 3 arbitrary beta nx={nx} ny={ny}")
    g = np.random.default_rng(nx + ny)
    beta = g.uniform(-0.9, 1.3, (4, ny, nx))       # arbitrary, not symmetric, mixed signs
    ub = g.standard_normal((ny, nx))
    A, bB = grid.beta_operator(nx, ny, beta, ub)
    Ainv = inverse.lu_inverse(A)
    assert np.max(np.abs(Ainv - Ainv.T)) > 1e-3  # genuinely non-symmetric
    # u = A^{-1} (rho + b_B) in the library's form u = -h^2 G rho + w: h = 1, G = -A^{-1}
    G = -Ainv
    w = apply.lift(Ainv, bB)
    N = G.shape[0]
    rho = g.uniform(-1, 1, (37, N))
    gv = g.standard_normal((37, N))
    with pinv.PoissonInverse.from_inverse(nx, ny, 1.0, G, None, ub, w) as op:
        u = host(op.apply(dev(rho), "fp64"))
        ref = Ainv @ (rho.T + bB[:, None])
        assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12
        lam = host(op.apply_adjoint(dev(gv), "fp64"))
        lam_ref = grad.adjoint(G, gv.T, 1.0)
        assert np.max(metrics.rel_l2_per_rhs(lam.T, lam_ref)) <= 1e-12

        op.quantize(24)
        ref8, _, _ = oracle_int8(G, 3, rho.T, 2, 1.0, w)
        assert np.array_equal(host(op.apply(dev(rho), "int8", 16)).T, ref8)
        qG, e = quant.quantize_rows(G, 3)
        qg, f = quant.quantize_cols(gv.T, 2, pre_exponent=e)
        ref_adj, _ = apply.integer_apply(qG.T, e, 3, qg, f, 2, 1.0, None, row_exponent=False)
        assert np.array_equal(host(op.apply_adjoint(dev(gv), "int8", 16)).T, ref_adj)


def _paper_beta(nx, ny, g):
    """beta_d = 4 eps_f / (sum of the node's four face eps_f), eps random positive:
    the row-normalised conservative operator (an M-matrix, rows summing to 0)."""
    eps = g.uniform(0.5, 2.0, (ny, nx))
    beta = np.zeros((4, ny, nx))
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            ef = [0.5 * (eps[i, j] + eps[i + di, j + dj]) for (di, dj) in grid.BETA_DIRECTIONS]
            beta[:, i, j] = 4.0 * np.array(ef) / sum(ef)
    return beta


@pytest.mark.parametrize("nx,ny,kind", [(12, 9, "paper"), (40, 31, "paper"), (37, 22, "dominant")])
def test_gpu_lu_build_matches_oracle(torch, nx, ny, kind):
    """The GPU LU build of Eq. 3's matrix (partial pivoting) against the oracle's
    pivoted LU inverse: the paper's row-normalised coefficients, and a strictly
    diagonally dominant non-symmetric set with mixed signs; N = 70, 1102, 700
    (ragged last 64-block); FP64 apply and adjoint on the built op."""
    from paper_1602_00001_amd import pinv
    announce(f"Eq. 3 GPU LU build nx={nx} ny={ny} {kind}")
    g = np.random.default_rng(nx * ny)
    beta = _paper_beta(nx, ny, g) if kind == "paper" else g.uniform(-0.9, 0.9, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    A, bB = grid.beta_operator(nx, ny, beta, ub)
    Ainv = inverse.lu_inverse(A)
    assert np.max(np.abs(Ainv - Ainv.T)) > 1e-6
    w = apply.lift(Ainv, bB)
    N = A.shape[0]
    rho = g.uniform(-1, 1, (29, N))
    gv = g.standard_normal((29, N))
    with pinv.PoissonInverse.build_beta(nx, ny, beta, ub) as op:
        info = op.info()
        assert info["beta"] == 1 and info["h"] == 1.0 and info["n"] == N
        Gg, wg = op.export_inverse()
        assert np.max(np.abs(Gg + Ainv)) <= 1e-12 * np.max(np.abs(Ainv))
        assert np.max(np.abs(wg - w)) <= 1e-12 * np.max(np.abs(w))
        u = host(op.apply(dev(rho), "fp64"))
        ref = Ainv @ (rho.T + bB[:, None])
        assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12
        lam = host(op.apply_adjoint(dev(gv), "fp64"))
        assert np.max(metrics.rel_l2_per_rhs(lam.T, grad.adjoint(-Ainv, gv.T, 1.0))) <= 1e-12
        with pytest.raises(pinv.PinvError) as ei:
            op.grad_eps(dev(rho[:1]), dev(rho[:1]))
        assert ei.value.status == pinv.E_UNSUPPORTED


def test_gpu_lu_build_needs_row_exchanges(torch):
    """A = [[1, -1, 0], [-1, 1, -1], [0, -1, 1]] (3 interior nodes in a row, all
    four inner coefficients 4): elimination in natural order meets a zero second
    pivot, but A is regular (det = -1) with the integer inverse -M,
    M = [[0, 1, 1], [1, 1, 1], [1, 1, 0]]; with row exchanges every operation is
    on small integers, so G = -A^{-1} = M exactly."""
    from paper_1602_00001_amd import pinv
    announce("Eq. 3 GPU LU build with a row exchange (3 unknowns)")
    nx, ny = 5, 3
    beta = np.zeros((4, ny, nx))
    beta[3, 1, 1] = 4.0     # (1,1) -> (1,2)
    beta[2, 1, 2] = 4.0     # (1,2) -> (1,1)
    beta[3, 1, 2] = 4.0     # (1,2) -> (1,3)
    beta[2, 1, 3] = 4.0     # (1,3) -> (1,2)
    A, _ = grid.beta_operator(nx, ny, beta)
    assert np.array_equal(A, np.array([[1.0, -1.0, 0.0], [-1.0, 1.0, -1.0], [0.0, -1.0, 1.0]]))
    M = np.array([[0.0, 1.0, 1.0], [1.0, 1.0, 1.0], [1.0, 1.0, 0.0]])
    with pinv.PoissonInverse.build_beta(nx, ny, beta) as op:
        Gg, _ = op.export_inverse()
    assert np.array_equal(Gg, M)


@pytest.mark.parametrize("nx,ny,lo,hi", [(40, 31, -3.0, 3.0), (37, 22, -4.0, 4.0), (12, 9, -4.0, 4.0)])
def test_gpu_lu_build_mixed_sign_coefficients(torch, nx, ny, lo, hi):
    """Coefficients uniform in (lo, hi), neither dominant nor of one sign: the
    factorization needs row exchanges (without them the pivots fall to 1e-3 and
    the entries grow by up to ~900).  The GPU inverse against the oracle's
    pivoted LU inverse within 64 cond(A) eps (both are backward stable), and its
    residual |A X - I| within 1e-12 |A| |X| (max norms); the lift likewise."""
    from paper_1602_00001_amd import pinv
    announce(f"Eq. 3 GPU LU build, mixed-sign beta in ({lo}, {hi}) nx={nx} ny={ny}")
    g = np.random.default_rng(nx * ny + 7)
    beta = g.uniform(lo, hi, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    A, bB = grid.beta_operator(nx, ny, beta, ub)
    Ainv = inverse.lu_inverse(A)
    cond = np.linalg.norm(A, 2) * np.linalg.norm(Ainv, 2)
    tol = 64.0 * cond * np.finfo(np.float64).eps
    w = apply.lift(Ainv, bB)
    with pinv.PoissonInverse.build_beta(nx, ny, beta, ub) as op:
        Gg, wg = op.export_inverse()
    X = -Gg
    assert np.max(np.abs(X - Ainv)) <= tol * np.max(np.abs(Ainv))
    assert np.max(np.abs(wg - w)) <= tol * np.max(np.abs(w))
    res = A @ X - np.eye(A.shape[0])
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(A)) * np.max(np.abs(X)) * A.shape[0] ** 0.5


def test_gpu_lu_build_reports_a_zero_pivot(torch):
    """A = [[1, -1, 0], [-1, 1, 0], [0, 0, 1]] (3 interior nodes in a row, two
    coefficients of 4) is singular: after the first column (rows 0 and 1 tie,
    row 0 is kept) the second column has no non-zero candidate, reported as
    PINV_E_NOT_SPD."""
    from paper_1602_00001_amd import pinv
    announce("Eq. 3 GPU LU build of a singular matrix -> E_NOT_SPD")
    nx, ny = 5, 3
    beta = np.zeros((4, ny, nx))
    beta[3, 1, 1] = 4.0     # (1,1) -> (1,2)
    beta[2, 1, 2] = 4.0     # (1,2) -> (1,1)
    A, _ = grid.beta_operator(nx, ny, beta)
    assert np.array_equal(A, np.array([[1.0, -1.0, 0.0], [-1.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    with pytest.raises(pinv.PinvError) as ei:
        pinv.PoissonInverse.build_beta(nx, ny, beta)
    assert ei.value.status == pinv.E_NOT_SPD


@pytest.mark.parametrize("nx,ny,R,with_ub", [(12, 9, 37, True), (40, 31, 5, False), (9, 8, 0, True)])
def test_grad_beta_matches_oracle(torch, nx, ny, R, with_ub):
    """dLoss/dbeta on a GPU-built Eq. 3 op against the oracle's formula on the
    same (u, lambda): 1 and 3 chunks of right-hand sides, R = 0; and the whole
    chain (GPU forward, adjoint, gradient) against central differences."""
    from paper_1602_00001_amd import pinv
    announce(f"grad_beta nx={nx} ny={ny} R={R} ub={with_ub}")
    g = np.random.default_rng(nx * ny + R)
    beta = g.uniform(0.2, 1.0, (4, ny, nx))
    ub = g.standard_normal((ny, nx)) if with_ub else None
    N = (nx - 2) * (ny - 2)
    u = g.standard_normal((R, N))
    lam = g.standard_normal((R, N))
    ref = grad.grad_beta(nx, ny, u.T, lam.T, ub)
    with pinv.PoissonInverse.build_beta(nx, ny, beta, ub) as op:
        got = host(op.grad_beta(dev(u), dev(lam)))
        assert got.shape == (4, ny, nx)
        if R == 0:
            assert np.all(got == 0.0)
            return
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        # the chain through the GPU forward and adjoint, against re-solved losses
        rho = g.standard_normal((3, N))
        sample = np.sort(g.choice(N, 11, replace=False))
        d = 0.01 * g.standard_normal((11, 3))
        uf = op.apply(dev(rho), "fp64")
        gu = grad.sampling_loss_grad_u(host(uf).T, sample, d)
        lf = op.apply_adjoint(dev(gu.T), "fp64")
        gb = host(op.grad_beta(uf, lf))

    def loss(b):
        A, bB = grid.beta_operator(nx, ny, b, ub)
        uu = np.linalg.solve(A, rho.T + bB[:, None])
        res = uu[sample] - d
        return float(np.sum(res * res))

    v = g.standard_normal((4, ny, nx))
    fd = grad.central_difference(loss, beta, v, 1e-6)
    assert abs(fd - float(np.sum(gb * v))) <= 1e-6 * abs(fd)


def _stencil(nx, ny, beta, X):
    """Eq. 3's matrix applied to the columns of X [N, R] without forming it:
    (A x)_p = x_p - sum_d beta_d(p) / 4 x_{q_d}, interior neighbours only."""
    my, mx = ny - 2, nx - 2
    R = X.shape[1]
    U = np.zeros((ny, nx, R))
    U[1:-1, 1:-1] = X.reshape(my, mx, R)
    out = X.reshape(my, mx, R).copy()
    for d, (di, dj) in enumerate(grid.BETA_DIRECTIONS):
        out -= 0.25 * beta[d, 1:-1, 1:-1, None] * U[1 + di:ny - 1 + di, 1 + dj:nx - 1 + dj]
    return out.reshape(my * mx, R)


def _boundary_rhs(nx, ny, beta, ub):
    """b_B[p] = sum_d beta_d(p) / 4 u_B(q_d) over the boundary neighbours."""
    B = np.array(ub, dtype=np.float64)
    B[1:-1, 1:-1] = 0.0
    out = np.zeros((ny - 2, nx - 2))
    for d, (di, dj) in enumerate(grid.BETA_DIRECTIONS):
        out += 0.25 * beta[d, 1:-1, 1:-1] * B[1 + di:ny - 1 + di, 1 + dj:nx - 1 + dj]
    return out.reshape(-1)


def test_stencil_helpers_match_the_oracle_operator():
    """The full-size test's matrix-free stencil and boundary term equal the
    oracle's dense Eq. 3 matrix and b_B on a small grid."""
    g = np.random.default_rng(5)
    nx, ny = 9, 7
    beta = g.uniform(-2.0, 2.0, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    A, bB = grid.beta_operator(nx, ny, beta, ub)
    assert np.array_equal(_stencil(nx, ny, beta, np.eye(A.shape[0])), A)
    assert np.allclose(_boundary_rhs(nx, ny, beta, ub), bB, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", ["paper", "mixed"])
def test_gpu_lu_build_full_size(torch, kind):
    """128 x 128 grid (N = 15876): the paper's row-normalised coefficients, and
    mixed-sign ones in (-3, 3) that need row exchanges.  No dense reference at
    this size: 18 columns of A^{-1} (first, last, 16 random) from the FP64
    apply of unit vectors satisfy A x = e_j to 1e-12 |A| |X| sqrt(N) (max
    norms), and the lift satisfies A w = b_B likewise."""
    import time
    from paper_1602_00001_amd import pinv
    nx = ny = 128
    announce(f"Eq. 3 GPU LU build at 128x128 ({kind})")
    g = np.random.default_rng(128)
    beta = _paper_beta(nx, ny, g) if kind == "paper" else g.uniform(-3.0, 3.0, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    N = (nx - 2) * (ny - 2)
    cols = np.concatenate([[0, N - 1], g.choice(np.arange(1, N - 1), 16, replace=False)])
    E = np.zeros((cols.size, N))
    E[np.arange(cols.size), cols] = 1.0
    t0 = time.perf_counter()
    with pinv.PoissonInverse.build_beta(nx, ny, beta, ub) as op:
        t_build = time.perf_counter() - t0
        u = host(op.apply(dev(E), "fp64"))
        w = host(op.apply(dev(np.zeros((1, N))), "fp64"))[0]     # -G 0 + w
    print(f"build_beta 128x128 {kind}: {t_build:.2f} s")
    X = (u - w[None, :]).T
    res = _stencil(nx, ny, beta, X) - E.T
    amax = 1.0 + 0.25 * np.max(np.sum(np.abs(beta[:, 1:-1, 1:-1]), axis=0))
    assert np.max(np.abs(res)) <= 1e-12 * amax * np.max(np.abs(X)) * N ** 0.5
    rw = _stencil(nx, ny, beta, w[:, None])[:, 0] - _boundary_rhs(nx, ny, beta, ub)
    assert np.max(np.abs(rw)) <= 1e-12 * amax * np.max(np.abs(w)) * N ** 0.5


def test_autograd_beta_matches_finite_differences(torch):
    """PinvSolveBeta (FP64 mode) on a GPU-built Eq. 3 op with mixed-sign
    coefficients: gradients of sum ||C u - d||^2 in rho and beta against
    central differences of the dense re-solved loss (1e-6)."""
    from paper_1602_00001_amd import pinv
    from paper_1602_00001_amd.autograd import PinvSolveBeta
    announce("autograd PinvSolveBeta vs central differences 11x9")
    nx, ny = 11, 9
    g = np.random.default_rng(913)
    beta = g.uniform(-2.0, 2.0, (4, ny, nx))
    ub = g.standard_normal((ny, nx))
    N = (nx - 2) * (ny - 2)
    rho = g.standard_normal((2, N))
    sample = np.sort(g.choice(N, 13, replace=False))
    d = 0.01 * g.standard_normal((13, 2))

    def loss(b, r):
        A, bB = grid.beta_operator(nx, ny, b, ub)
        uu = np.linalg.solve(A, r.T + bB[:, None])
        res = uu[sample] - d
        return float(np.sum(res * res))

    T = torch
    with pinv.PoissonInverse.build_beta(nx, ny, beta, ub) as op:
        rt = dev(rho).requires_grad_(True)
        bt = dev(beta).requires_grad_(True)
        u = PinvSolveBeta.apply(rt, bt, op, "fp64", 16)
        st = T.from_numpy(sample).cuda()
        dt = dev(d.T)
        L = T.sum((u[:, st] - dt) ** 2)
        L.backward()
        gr = host(rt.grad)
        gb = host(bt.grad)
    v = g.standard_normal((4, ny, nx))
    fd = grad.central_difference(lambda b: loss(b, rho), beta, v, 1e-6)
    assert abs(fd - float(np.sum(gb * v))) <= 1e-6 * abs(fd)
    w = g.standard_normal((2, N))
    fd = grad.central_difference(lambda r: loss(beta, r), rho, w, 1e-6)
    assert abs(fd - float(np.sum(gr * w))) <= 1e-6 * abs(fd)
