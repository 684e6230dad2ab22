"""Checkpoint round trip (pinv_save / pinv_load): an op written to a file and
read back holds bit for bit the same G, digit slices, row exponents and lift,
and gives bit-identical applies, adjoints and
permittivity gradients -- for a 2-D op with Dirichlet data (FP64 and slices),
a slices-only op, a 3-D op, a non-uniform-grid op and an Eq. 3 op."""

import numpy as np
import pytest

from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


def _same(a, b):
    return bool(a.shape == b.shape and np.array_equal(host(a), host(b)))


def test_round_trip_2d_fp64_and_slices(torch, pinv, tmp_path):
    nx, ny = 40, 33
    g = np.random.default_rng(44)
    h = 1.0 / (nx - 1)
    ub = g.standard_normal((ny, nx))
    eps = workloads.random_eps(nx, ny, g)
    N = (nx - 2) * (ny - 2)
    rho = dev(g.uniform(-1, 1, (7, N)))
    gv = dev(g.standard_normal((3, N)))
    path = tmp_path / "op2d.pinv"
    announce("checkpoint 2-D op with Dirichlet data, FP64 + 24-bit slices")
    with pinv.PoissonInverse.build(nx, ny, h, eps, ub) as op:
        op.quantize(24)
        op.set_int8_variant(16, 13)
        ref = {"fp64": op.apply(rho, "fp64"), "int8": op.apply(rho, "int8", 16),
               "adj8": op.apply_adjoint(gv, "int8", 16), "adj64": op.apply_adjoint(gv, "fp64")}
        ref["grad"] = op.grad_eps(ref["fp64"][:3], ref["adj64"])
        G0, w0 = op.export_inverse()
        Q0, e0 = op.export_quantized()
        info0 = op.info()
        op.save(path)
    assert path.stat().st_size > 8 * N * N
    with pinv.PoissonInverse.load(path) as op2:
        info = op2.info()
        for k in ("nx", "ny", "n", "h", "nz", "has_fp64", "int8_slices", "has_lift", "general", "beta"):
            assert info[k] == info0[k], k
        assert (op2.nx, op2.ny, op2.n) == (nx, ny, N)
        G1, w1 = op2.export_inverse()
        Q1, e1 = op2.export_quantized()
        assert np.array_equal(G0, G1) and np.array_equal(w0, w1)
        assert np.array_equal(Q0, Q1) and np.array_equal(e0, e1)
        assert _same(op2.apply(rho, "fp64"), ref["fp64"])
        assert _same(op2.apply(rho, "int8", 16), ref["int8"])
        assert _same(op2.apply_adjoint(gv, "int8", 16), ref["adj8"])
        adj64 = op2.apply_adjoint(gv, "fp64")
        assert _same(adj64, ref["adj64"])
        assert _same(op2.grad_eps(op2.apply(rho, "fp64")[:3], adj64), ref["grad"])
        # (the variant choice is saved too; any variant gives the same result)
        op2.set_int8_variant(16, 0)
        assert _same(op2.apply(rho, "int8", 16), ref["int8"])

        # slices only (FP64 G dropped): saved and loaded without G
        op2.quantize(16, keep_fp64=False)
        ref16 = op2.apply(rho, "int8", 16)
        p16 = tmp_path / "op2d_16.pinv"
        op2.save(p16)
    assert p16.stat().st_size < 8 * N * N
    with pinv.PoissonInverse.load(p16) as op3:
        assert op3.info()["has_fp64"] == 0 and op3.info()["int8_slices"] == 2
        assert _same(op3.apply(rho, "int8", 16), ref16)
        with pytest.raises(pinv.PinvError) as ei:
            op3.apply(rho, "fp64")
        assert ei.value.status == pinv.E_STATE


def test_round_trip_3d_general_beta(torch, pinv, tmp_path):
    g = np.random.default_rng(45)
    announce("checkpoint 3-D, non-uniform-grid and Eq. 3 ops")
    # 3-D, no Dirichlet data
    with pinv.PoissonInverse.build3d(9, 8, 7) as op:
        N = op.n
        rho = dev(g.uniform(-1, 1, (5, N)))
        ref = op.apply(rho, "fp64")
        op.save(tmp_path / "op3d.pinv")
    with pinv.PoissonInverse.load(tmp_path / "op3d.pinv") as op2:
        assert (op2.nx, op2.ny, op2.nz, op2.n) == (9, 8, 7, N)
        assert _same(op2.apply(rho, "fp64"), ref)
    # non-uniform grid, per-direction eps, Dirichlet data: the node
    # coordinates travel with the op (the gradient needs them)
    x = np.cumsum(g.uniform(0.5, 1.5, 14))
    y = np.cumsum(g.uniform(0.5, 1.5, 11))
    ex, ey = workloads.random_eps(14, 11, g), workloads.random_eps(14, 11, g)
    ub = g.standard_normal((11, 14))
    with pinv.PoissonInverse.build_general(x, y, ex, ey, ub) as op:
        N = op.n
        rho = dev(g.uniform(-1, 1, (4, N)))
        u = op.apply(rho, "fp64")
        lam = op.apply_adjoint(dev(g.standard_normal((4, N))), "fp64")
        gx, gy = op.grad_eps_general(u, lam)
        op.save(tmp_path / "opgen.pinv")
    with pinv.PoissonInverse.load(tmp_path / "opgen.pinv") as op2:
        assert op2.info()["general"] == 1
        assert _same(op2.apply(rho, "fp64"), u)
        gx2, gy2 = op2.grad_eps_general(u, lam)
        assert _same(gx2, gx) and _same(gy2, gy)
    # Eq. 3 with arbitrary positive coefficients (a non-symmetric operator)
    beta = g.uniform(0.5, 1.5, (4, 10, 12))
    with pinv.PoissonInverse.build_beta(12, 10, beta) as op:
        N = op.n
        rho = dev(g.uniform(-1, 1, (6, N)))
        u = op.apply(rho, "fp64")
        gb = op.grad_beta(u, op.apply_adjoint(rho, "fp64"))
        op.save(tmp_path / "opbeta.pinv")
    with pinv.PoissonInverse.load(tmp_path / "opbeta.pinv") as op2:
        assert op2.info()["beta"] == 1
        assert _same(op2.apply(rho, "fp64"), u)
        assert _same(op2.grad_beta(u, op2.apply_adjoint(rho, "fp64")), gb)
