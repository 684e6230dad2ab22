"""Non-uniform tensor grids with permittivity per direction (Eq. 1's eps_i):
the GPU build against the oracle's finite-volume operator (G = K^{-1} diag(A)
and the lift), the uniform special case against the standard build bit for
bit, the FP64 and int8 applies, the per-direction eps-gradients against the
oracle's face loop (the uniform-grid gradient entry point refuses these ops)."""

import numpy as np
import pytest

from oracle import apply, grad, grid, inverse, metrics
from tests.gpu_util import announce, dev, host, oracle_int8, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


def _coords(g, n):
    return np.sort(np.concatenate([[0.0, 1.0], g.uniform(0.0, 1.0, n - 2)]))


@pytest.mark.parametrize("nx,ny,aniso", [(3, 3, True), (14, 11, True), (40, 33, True), (21, 18, False)])
def test_general_build_matches_oracle(torch, pinv, nx, ny, aniso):
    """aniso False: one field for both directions (eps_y omitted)."""
    announce(f"general build nx={nx} ny={ny} anisotropic={aniso}")
    g = np.random.default_rng(nx * 100 + ny)
    x, y = _coords(g, nx), _coords(g, ny)
    ex = g.uniform(0.3, 3.0, (ny, nx))
    ey = g.uniform(0.3, 3.0, (ny, nx)) if aniso else None
    ub = g.standard_normal((ny, nx))
    K, bB, A = grid.conservative_operator_general(x, y, ex, ey, ub)
    Ginv = inverse.lu_inverse(K)
    Gp = Ginv * A[None, :]
    w = apply.lift(Ginv, bB)
    with pinv.PoissonInverse.build_general(x, y, ex, ey, ub) as op:
        assert op.info()["general"] == 1
        Gg, wg = op.export_inverse()
        assert np.max(np.abs(Gg - Gp)) <= 1e-12 * np.max(np.abs(Gp))
        assert np.max(np.abs(wg - w)) <= 1e-12 * np.max(np.abs(w))
        rho = g.uniform(-1, 1, (9, op.n))
        u = host(op.apply(dev(rho), "fp64"))
        ref = np.linalg.solve(K, -A[:, None] * rho.T + bB[:, None])
        assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12
        with pytest.raises(pinv.PinvError) as ei:
            op.grad_eps(dev(rho[:2]), dev(rho[:2]), out=torch.empty((ny, nx), dtype=torch.float64, device="cuda"))
        assert ei.value.status == pinv.E_UNSUPPORTED


def test_uniform_general_build_equals_standard_build(torch, pinv):
    """Power-of-two spacing: every face weight and area is exact, so the general
    build is h^2 times the standard build, bit for bit."""
    nx, ny, h = 17, 9, 0.125
    g = np.random.default_rng(5)
    eps = g.uniform(0.5, 2.0, (ny, nx))
    ub = g.standard_normal((ny, nx))
    with pinv.PoissonInverse.build_general(np.arange(nx) * h, np.arange(ny) * h, eps, eps, ub) as og, \
            pinv.PoissonInverse.build(nx, ny, h, eps, ub) as os_:
        Gg, wg = og.export_inverse()
        Gs, ws = os_.export_inverse()
    assert np.array_equal(Gg, Gs * (h * h))
    assert np.array_equal(wg, ws)


def test_general_int8_apply(torch, pinv):
    """Int8 on a general inverse: bit for bit against the oracle's integer apply
    on the oracle's G (imported), and within the 24-bit envelope on the
    GPU-built op."""
    g = np.random.default_rng(77)
    nx, ny = 30, 26
    x, y = _coords(g, nx), _coords(g, ny)
    ex = g.uniform(0.3, 3.0, (ny, nx))
    K, bB, A = grid.conservative_operator_general(x, y, ex)
    Gp = inverse.lu_inverse(K) * A[None, :]
    rho = g.uniform(-1, 1, (140, Gp.shape[0]))
    ref, _, _ = oracle_int8(Gp, 3, rho.T, 2, 1.0)
    with pinv.PoissonInverse.from_inverse(nx, ny, 1.0, Gp) as op:
        op.quantize(24)
        assert np.array_equal(host(op.apply(dev(rho), "int8", 16)).T, ref)
    u64 = apply.plain_apply(Gp, rho.T, 1.0, None)
    with pinv.PoissonInverse.build_general(x, y, ex) as op:
        op.quantize(24)
        u = host(op.apply(dev(rho), "int8", 16))
    assert np.max(metrics.rel_l2_per_rhs(u.T, u64)) <= 2e-4


@pytest.mark.parametrize("nx,ny,R,with_ub,split", [(14, 11, 5, True, True), (29, 23, 37, True, True),
                                                   (19, 16, 20, False, False), (9, 8, 0, True, True)])
def test_grad_eps_general_matches_oracle(torch, pinv, nx, ny, R, with_ub, split):
    """GPU per-direction gradients (or their sum) on a GPU-built non-uniform op
    against the oracle on the same (u, lambda): 72-667 nodes (ragged 256-node
    workgroups), 1 or 3 chunks of right-hand sides, R = 0."""
    announce(f"grad_eps_general nx={nx} ny={ny} R={R} ub={with_ub} split={split}")
    g = np.random.default_rng(nx * ny + R)
    x, y = _coords(g, nx), _coords(g, ny)
    ex = g.uniform(0.3, 3.0, (ny, nx))
    ey = g.uniform(0.3, 3.0, (ny, nx))
    ub = g.standard_normal((ny, nx)) if with_ub else None
    N = (nx - 2) * (ny - 2)
    u = g.standard_normal((R, N))
    lam = g.standard_normal((R, N))
    rx, ry = grad.grad_eps_general(x, y, u.T, lam.T, ub)
    with pinv.PoissonInverse.build_general(x, y, ex, ey, ub) as op:
        out = op.grad_eps_general(dev(u), dev(lam), split=split)
        if split:
            gx, gy = host(out[0]), host(out[1])
        else:
            gs = host(out)
    if R == 0:
        assert np.all(gx == 0.0) and np.all(gy == 0.0)
    elif split:
        assert np.max(np.abs(gx - rx)) <= 1e-12 * np.max(np.abs(rx))
        assert np.max(np.abs(gy - ry)) <= 1e-12 * np.max(np.abs(ry))
    else:
        ref = rx + ry
        assert np.max(np.abs(gs - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_grad_eps_general_refuses_uniform_ops(torch, pinv):
    announce("grad_eps_general on a uniform op -> E_UNSUPPORTED")
    with pinv.PoissonInverse.build(6, 5, 0.2) as op:
        z = dev(np.zeros((1, op.n)))
        with pytest.raises(pinv.PinvError) as ei:
            op.grad_eps_general(z, z)
        assert ei.value.status == pinv.E_UNSUPPORTED


def test_autograd_general_matches_finite_differences(torch, pinv):
    """PinvSolveGeneral on a GPU-built non-uniform op (FP64 mode): gradients of
    sum ||C u - d||^2 in rho, eps_x and eps_y against central differences of
    the oracle's re-solved finite-volume system."""
    from paper_1602_00001_amd.autograd import PinvSolveGeneral
    announce("autograd PinvSolveGeneral vs central differences 15x12")
    g = np.random.default_rng(29)
    nx, ny = 15, 12
    x, y = _coords(g, nx), _coords(g, ny)
    ex = g.uniform(0.5, 2.0, (ny, nx))
    ey = g.uniform(0.5, 2.0, (ny, nx))
    N = (nx - 2) * (ny - 2)
    rho = g.standard_normal((3, N))
    sample = np.sort(g.choice(N, 25, replace=False))
    d = 0.01 * g.standard_normal((25, 3))
    with pinv.PoissonInverse.build_general(x, y, ex, ey) as op:
        rt = dev(rho).requires_grad_(True)
        xt = dev(ex).requires_grad_(True)
        yt = dev(ey).requires_grad_(True)
        u = PinvSolveGeneral.apply(rt, xt, yt, op, "fp64", 16)
        idx = torch.from_numpy(sample).cuda()
        loss = ((u[:, idx] - dev(d.T)) ** 2).sum()
        loss.backward()
        gr, gx, gy = host(rt.grad), host(xt.grad), host(yt.grad)

    def lossf(a, b, r):
        K, _, A = grid.conservative_operator_general(x, y, a, b)
        uu = np.linalg.solve(K, -A[:, None] * r.T)
        res = uu[sample] - d
        return float(np.sum(res * res))

    v = g.standard_normal((ny, nx))
    fd = grad.central_difference(lambda a: lossf(a, ey, rho), ex, v, 1e-6)
    assert abs(fd - float(np.sum(gx * v))) <= 1e-6 * abs(fd)
    fd = grad.central_difference(lambda b: lossf(ex, b, rho), ey, v, 1e-6)
    assert abs(fd - float(np.sum(gy * v))) <= 1e-6 * abs(fd)
    vr = g.standard_normal(rho.shape)
    fd = grad.central_difference(lambda r: lossf(ex, ey, r), rho, vr, 1e-6)
    assert abs(fd - float(np.sum(gr * vr))) <= 1e-6 * abs(fd)
