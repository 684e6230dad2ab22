"""The symmetric-packed FP64 form (upper-triangle 64 x 64 blocks, one pass
over half the bytes of G): against the oracle's FP64 product for inverses of
1 to 1178 unknowns (a single partial block, exact block multiples, ragged last
blocks), 1 to 11 right-hand sides (one and two passes of up to 8), strided
vectors, the lift; the adjoint (G symmetric); GPU-built 2-D and 3-D ops; the
refusal for non-symmetric inverses."""

import numpy as np
import pytest

from oracle import apply, grid, inverse, metrics
from tests.gpu_util import announce, dev, host, oracle_inverse, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


@pytest.mark.parametrize("nx,ny", [(3, 3), (10, 10), (12, 9), (21, 17), (40, 33)])
@pytest.mark.parametrize("nrhs", [1, 3, 8, 11])
def test_sym_apply_matches_oracle(torch, pinv, nx, ny, nrhs):
    announce(f"apply fp64_sym nx={nx} ny={ny} nrhs={nrhs}")
    g = np.random.default_rng(nx * ny + nrhs)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    ub = g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, eps, ub)
    N = G.shape[0]
    rho = g.uniform(-1, 1, (nrhs, N + 5))
    ref = apply.plain_apply(G, rho[:, :N].T, h, w)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, eps, ub, w) as op:
        op.prepare_split("fp64_sym")
        assert op.info()["has_sym"] == 1
        out = torch.full((nrhs, N + 2), float("nan"), dtype=torch.float64, device="cuda")[:, :N]
        op.apply(dev(rho)[:, :N], "fp64_sym", out=out)
        u = host(out)
        assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12
        lam = host(op.apply_adjoint(dev(rho[:, :N]), "fp64_sym"))
        assert np.max(metrics.rel_l2_per_rhs(lam.T, -(h * h) * (G.T @ rho[:, :N].T))) <= 1e-12


def test_sym_on_gpu_built_ops(torch, pinv):
    """2-D and 3-D inverses built on the GPU are accepted; the packed copy
    outlives the FP64 G (freed by quantize(keep_fp64=False))."""
    announce("fp64_sym on GPU-built 2-D and 3-D ops")
    g = np.random.default_rng(3)
    nx, ny = 37, 29
    h = 1.0 / (nx - 1)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    G, _, _ = oracle_inverse(nx, ny, eps)
    rho = g.uniform(-1, 1, (6, G.shape[0]))
    ref = apply.plain_apply(G, rho.T, h)
    with pinv.PoissonInverse.build(nx, ny, h, eps) as op:
        op.prepare_split("fp64_sym")
        op.quantize(16, keep_fp64=False)
        u = host(op.apply(dev(rho), "fp64_sym"))
        assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12
    n3 = 9
    K, _ = grid.conservative_operator_3d(n3, n3, n3)
    G3 = inverse.lu_inverse(K)
    r3 = g.uniform(-1, 1, (2, G3.shape[0]))
    with pinv.PoissonInverse.build3d(n3, n3, n3, 0.125) as op:
        op.prepare_split("fp64_sym")
        u = host(op.apply(dev(r3), "fp64_sym"))
    assert np.max(metrics.rel_l2_per_rhs(u.T, apply.plain_apply(G3, r3.T, 0.125))) <= 1e-12


def test_sym_refuses_non_symmetric_inverses(torch, pinv):
    announce("fp64_sym refused for non-symmetric inverses; E_STATE before prepare")
    g = np.random.default_rng(4)
    x = np.sort(np.concatenate([[0.0, 1.0], g.uniform(0, 1, 10)]))
    with pinv.PoissonInverse.build_general(x, x, g.uniform(0.5, 2.0, (12, 12))) as op:
        with pytest.raises(pinv.PinvError) as ei:
            op.prepare_split("fp64_sym")
        assert ei.value.status == pinv.E_UNSUPPORTED
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(dev(np.ones((1, op.n))), "fp64_sym")
        assert ei.value.status == pinv.E_STATE
    beta = g.uniform(0.2, 0.9, (4, 8, 9))
    with pinv.PoissonInverse.build_beta(9, 8, beta) as op:
        with pytest.raises(pinv.PinvError) as ei:
            op.prepare_split("fp64_sym")
        assert ei.value.status == pinv.E_UNSUPPORTED


def test_sym_batched_equals_per_request(torch, pinv):
    """apply_batched in the packed mode runs each request as a single apply."""
    announce("apply_batched fp64_sym")
    g = np.random.default_rng(12)
    ops, reqs = [], []
    try:
        for (nx, ny) in ((14, 11), (23, 19)):
            G, _, _ = oracle_inverse(nx, ny)
            op = pinv.PoissonInverse.from_inverse(nx, ny, 1.0 / (nx - 1), G)
            op.prepare_split("fp64_sym")
            ops.append((op, G))
        for k in range(6):
            op, G = ops[k % 2]
            rho = dev(g.uniform(-1, 1, (1 + k, op.n)))
            reqs.append((op, rho, torch.empty_like(rho), G))
        pinv.apply_batched([(op, rho, u) for (op, rho, u, _) in reqs], "fp64_sym")
        for (op, rho, u, G) in reqs:
            assert np.array_equal(host(u), host(op.apply(rho, "fp64_sym")))
            ref = apply.plain_apply(G, host(rho).T, op.h)
            assert np.max(metrics.rel_l2_per_rhs(host(u).T, ref)) <= 1e-12
    finally:
        for op, _ in ops:
            op.close()
