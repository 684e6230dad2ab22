"""Eq. 3 with arbitrary (non-symmetric) neighbour coefficients: the inverse is
computed on the host ("any standard matrix inversion method") and imported;
the apply and the adjoint then run the same GPU kernels.  The adjoint must be
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
