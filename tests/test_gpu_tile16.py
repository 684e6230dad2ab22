"""16-bit fixed point with 64 x 64 tile scales (storage variant for few
right-hand sides): the GPU quantiser bit for bit against the oracle's
quantize_tiles, the GPU apply against the oracle's tile_apply on the same
integers (different summation order: 1e-12), and at 126^2 sampled row blocks
against the closed-form inverse plus the 1e-4 accuracy bound."""

import numpy as np
import pytest

from oracle import apply, inverse, metrics, quant
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _decaying(N, g):
    """Non-symmetric test matrix whose magnitude decays away from the diagonal
    at different rates above and below it, so tile exponents differ across
    tiles and the table is not symmetric."""
    d = np.subtract.outer(np.arange(N), np.arange(N)).astype(np.float64)
    return g.standard_normal((N, N)) * np.where(d > 0, np.exp(-d / 40.0), np.exp(d / 9.0))


@pytest.mark.parametrize("nx,ny", [(10, 9), (40, 31), (66, 66)])
def test_tile16_quantiser_bit_exact(torch, nx, ny):
    """N = 56, 1102, 4096: ragged and whole last tiles."""
    from paper_1602_00001_amd import pinv
    announce(f"tile16 quantiser nx={nx} ny={ny}")
    N = (nx - 2) * (ny - 2)
    G = _decaying(N, np.random.default_rng(N))
    q_ref, e_ref = quant.quantize_tiles(G, 2, 64)
    assert np.max(np.abs(q_ref)) <= quant.max_mag(2)
    with pinv.PoissonInverse.from_inverse(nx, ny, 0.1, G) as op:
        op.prepare_split("fix16_tile")
        assert op.info()["has_tile16"] == 1
        q, e = op.export_tile16()
    assert np.array_equal(e, e_ref)
    assert e.shape[0] == 1 or not np.array_equal(e, e.T)
    assert np.array_equal(q.astype(np.int64), q_ref)


@pytest.mark.parametrize("nx,ny,R,lift,pad", [(10, 9, 1, False, 0), (40, 31, 3, True, 5), (40, 31, 9, True, 0),
                                               (66, 66, 4, False, 3), (35, 20, 2, True, 1)])
def test_tile16_apply_matches_oracle(torch, nx, ny, R, lift, pad):
    """u = -h^2/M sum_b 2^e q rho + w against the oracle on the oracle's own
    integers: 1-9 right-hand sides (chunks of 4 and a ragged chunk), strided
    vectors (ld = N + pad), with and without a lift; N = 56 (only the bounded
    step), 1102, 4096 (whole 512-column steps), 594; and the adjoint
    lambda = -h^2 G^T g on the transposed integers and exponents."""
    from paper_1602_00001_amd import pinv
    announce(f"tile16 apply nx={nx} ny={ny} R={R} lift={lift} pad={pad}")
    N = (nx - 2) * (ny - 2)
    g = np.random.default_rng(N + R)
    G = _decaying(N, g)
    h = 0.37
    ub = g.standard_normal((ny, nx)) if lift else None
    w = g.standard_normal(N) if lift else None
    q, e = quant.quantize_tiles(G, 2, 64)
    rho = g.uniform(-1, 1, (N, R))
    ref = apply.tile_apply(q, e, 2, 64, rho, h, w)
    X = np.zeros((R, N + pad))
    X[:, :N] = rho.T
    gv = g.standard_normal((N, R))
    ref_adj = apply.tile_apply(q.T, e.T, 2, 64, gv, h)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.prepare_split("fix16_tile")
        u = host(op.apply(dev(X)[:, :N], "fix16_tile"))
        lam = host(op.apply_adjoint(dev(gv.T), "fix16_tile"))
    assert np.max(np.abs(u.T - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the adjoint is the exact transpose of the rounded matrix (the oracle's
    # transposed integers and exponents); on these non-symmetric matrices the
    # forward copy would miss by far more
    assert np.max(np.abs(lam.T - ref_adj)) <= 1e-12 * np.max(np.abs(ref_adj))
    assert np.max(np.abs(apply.tile_apply(q, e, 2, 64, gv, h) - ref_adj)) > 1e-3 * np.max(np.abs(ref_adj))


def test_tile16_requires_prepare(torch):
    from paper_1602_00001_amd import pinv
    announce("tile16 apply before prepare -> E_STATE")
    G = _decaying(56, np.random.default_rng(3))
    with pinv.PoissonInverse.from_inverse(10, 9, 0.1, G) as op:
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(dev(np.ones((1, 56))), "fix16_tile")
        assert ei.value.status == pinv.E_STATE
        with pytest.raises(pinv.PinvError) as ei:
            op.export_tile16()
        assert ei.value.status == pinv.E_STATE


def test_tile16_full_size_126(torch):
    """128 x 128 grid (N = 15876), GPU-built inverse, 4 uniform right-hand
    sides: (a) relative L2 error against the closed-form solve <= 1e-4 (the
    accuracy bound the variant exists for); (b) the tile exponents and 64 rows
    of u in two sampled row blocks against the oracle's tile quantisation and
    tile_apply of the closed-form inverse's rows: the exponents equal, u within
    the effect of a one-unit change of every integer (the two inverses differ
    by rounding, which can move a product across a rounding boundary)."""
    from paper_1602_00001_amd import pinv
    announce("tile16 at 126^2 interior, R = 4")
    nx = ny = 128
    N = 126 * 126
    h = 1.0 / 127
    g = np.random.default_rng(126)
    rho = g.uniform(-1, 1, (N, 4))
    with pinv.PoissonInverse.build(nx, ny, h) as op:
        op.prepare_split("fix16_tile")
        u = host(op.apply(dev(rho.T), "fix16_tile")).T
        _, e = op.export_tile16()
    T = e.shape[0]
    M = quant.max_mag(2)
    for a in (0, 131):
        rows = np.arange(a * 64, min(N, (a + 1) * 64))
        Gb = inverse.dst_inverse_rows(nx, ny, rows)
        qb, eb = quant.quantize_tiles(Gb, 2, 64)
        assert np.array_equal(e[a], eb[0])
        ub_ = apply.tile_apply(qb, eb, 2, 64, rho, h)
        scale = np.repeat(np.ldexp(1.0, eb[0]), 64)[:N]
        bound = h * h / M * (scale @ np.abs(rho)) * (1 + 1e-9) + 1e-12 * np.max(np.abs(ub_))
        assert np.all(np.abs(u[rows] - ub_) <= bound[None, :])
    # (a) accuracy against the closed-form solve, applied through the DST
    # basis: G rho = Sy^T (inv o (Sy rho Sx^T)) Sx per right-hand side, the
    # same expansion as the oracle's closed-form rows
    Sy, ly = inverse.dst_basis(126)
    Sx, lx = inverse.dst_basis(126)
    inv = 1.0 / (ly[:, None] + lx[None, :])
    ref = np.stack([(Sy.T @ (inv * (Sy @ rho[:, r].reshape(126, 126) @ Sx.T)) @ Sx).reshape(-1)
                    for r in range(4)], axis=1) * -(h * h)
    rows = np.arange(0, N, 97)
    assert np.max(np.abs(ref[rows] + (h * h) * (inverse.dst_inverse_rows(nx, ny, rows) @ rho))) \
        <= 1e-12 * np.max(np.abs(ref))
    rel = metrics.rel_l2_per_rhs(u, ref)
    print(f"tile16 126^2 rel L2 per RHS: {rel}")
    assert np.max(rel) <= 1e-4
    assert T == 249
