"""GPU parity of the HIP path with the CPU oracle, through the C-ABI, at sizes
the oracle finishes in seconds (several tiles and ragged tails)."""

import numpy as np
import pytest

from oracle import apply, grad, metrics, quant, split
from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, check_split_solve, dev, host, oracle_int8, oracle_inverse, require_gpu

pytestmark = pytest.mark.gpu

# (nx, ny): N = 1, one partial tile, several tiles with ragged tails, non-square
SIZES = [(3, 3), (12, 9), (32, 32), (50, 37), (66, 66)]


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


# ---------------------------------------------------------------- build (steps 1-2)

@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("kind", ["one", "sincos", "random"])
def test_build_inverse_matches_oracle(torch, pinv, nx, ny, kind):
    announce(f"build_inverse nx={nx} ny={ny} eps={kind}")
    g = np.random.default_rng(nx * 100 + ny)
    eps = {"one": None, "random": workloads.random_eps(nx, ny, g),
           "sincos": 1.0 + 0.5 * np.sin(2 * np.pi * workloads.coords(max(nx, ny))[0][:ny, :nx])}[kind]
    ub = None if kind == "one" else g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, eps, ub)
    with pinv.PoissonInverse.build(nx, ny, h, eps, ub) as op:
        Gg, wg = op.export_inverse()
        assert np.linalg.norm(Gg - G) <= 1e-12 * np.linalg.norm(G)
        if ub is not None:
            assert np.linalg.norm(wg - w) <= 1e-12 * np.linalg.norm(w)
            assert op.info()["has_lift"] == 1
        else:
            assert np.all(wg == 0)


def test_build_rejects_non_spd(torch, pinv):
    announce("build_inverse negative eps -> E_NOT_SPD")
    n = 20
    eps = np.ones((n, n))
    eps[5:15, 5:15] = -3.0
    with pytest.raises(pinv.PinvError) as ei:
        pinv.PoissonInverse.build(n, n, 0.05, eps)
    assert ei.value.status == pinv.E_NOT_SPD


# ---------------------------------------------------------------- FP64 apply (step 3)

@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("nrhs", [1, 3, 5, 130])
def test_fp64_apply_matches_oracle(torch, pinv, nx, ny, nrhs):
    announce(f"apply fp64 nx={nx} ny={ny} nrhs={nrhs}")
    g = np.random.default_rng(7)
    ub = g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, None, ub)
    rho = g.uniform(-1, 1, (nrhs, G.shape[0]))
    ref = apply.plain_apply(G, rho.T, h, w)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        u = host(op.apply(dev(rho), "fp64"))
    assert np.max(metrics.rel_l2_per_rhs(u.T, ref)) <= 1e-12


def test_fp64_apply_strided_and_empty(torch, pinv):
    announce("apply fp64 strided ld and nrhs=0")
    nx, ny, h = 21, 17, 0.05
    G, _, _ = oracle_inverse(nx, ny)
    N = G.shape[0]
    rho = np.random.default_rng(1).standard_normal((9, N + 7))
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        r = dev(rho)[:, :N]                   # row stride N + 7
        out = torch.zeros((9, N + 3), dtype=torch.float64, device="cuda")[:, :N]
        op.apply(r, "fp64", out=out)
        u = host(out)
        assert np.max(metrics.rel_l2_per_rhs(u.T, apply.plain_apply(G, rho[:, :N].T, h))) <= 1e-12
        empty = torch.empty((0, N), dtype=torch.float64, device="cuda")
        assert op.apply(empty, "fp64").shape == (0, N)
        with pytest.raises(pinv.PinvError):
            op.apply(r, "int8")              # not quantised yet -> E_STATE


# ---------------------------------------------------------------- INT8 quantised apply

@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("bits", [8, 16, 24])
def test_quantize_inverse_bit_exact(torch, pinv, nx, ny, bits):
    announce(f"quantize_inverse nx={nx} ny={ny} bits={bits}")
    h = 1.0 / (max(nx, ny) - 1)
    G, _, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, np.random.default_rng(3)))
    S = bits // 8
    q, e = quant.quantize_rows(G, S)
    digits = quant.balanced_digits(q, S)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.quantize(bits)
        Qg, eg = op.export_quantized()
    assert np.array_equal(eg, e)
    assert np.array_equal(Qg.astype(np.int64), digits)


@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("bits,rho_bits", [(8, 8), (16, 16), (24, 16), (24, 24), (8, 24), (16, 8)])
def test_int8_apply_bit_exact(torch, pinv, nx, ny, bits, rho_bits):
    announce(f"apply int8 nx={nx} ny={ny} bits={bits} rho_bits={rho_bits}")
    g = np.random.default_rng(nx + bits + rho_bits)
    ub = g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, None, ub)
    N = G.shape[0]
    rho = g.uniform(-1, 1, (133, N))
    rho[5] = 0.0                                   # an all-zero right-hand side
    rho[6] *= 1e-3
    ref, _, _ = oracle_int8(G, bits // 8, rho.T, rho_bits // 8, h, w)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.quantize(bits)
        u = host(op.apply(dev(rho), "int8", rho_bits))
    assert np.array_equal(u.T, ref)


def test_apply_with_a_very_large_row_stride(torch, pinv):
    """Right-hand sides 2^25 + 16 doubles apart (127 strides exceed 2^32
    elements): the FP64 GEMM and the int8 path address them in 64 bits."""
    announce("apply with row stride 2^25 + 16 (fp64 GEMM, int8)")
    nx, ny = 12, 9
    h = 1.0 / (nx - 1)
    G, _, _ = oracle_inverse(nx, ny)
    N = G.shape[0]
    ld = (1 << 25) + 16
    g = np.random.default_rng(21)
    rho = g.uniform(-1, 1, (5, N))
    big = torch.zeros((5, ld), dtype=torch.float64, device="cuda")
    big[:, :N] = dev(rho)
    out = torch.zeros((5, ld), dtype=torch.float64, device="cuda")
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.apply(big[:, :N], "fp64", out=out[:, :N])
        u = host(out[:, :N])
        assert np.max(metrics.rel_l2_per_rhs(u.T, apply.plain_apply(G, rho.T, h))) <= 1e-12
        op.quantize(24)
        op.apply(big[:, :N], "int8", 16, out=out[:, :N])
        ref, _, _ = oracle_int8(G, 3, rho.T, 2, h)
        assert np.array_equal(host(out[:, :N]).T, ref)
    del big, out


@pytest.mark.parametrize("nx,ny", [(3, 3), (12, 9), (40, 33)])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 7, 16, 17])
@pytest.mark.parametrize("bits,rho_bits", [(24, 16), (16, 16), (8, 24), (24, 24)])
def test_int8_few_rhs_bit_exact(torch, pinv, nx, ny, nrhs, bits, rho_bits):
    """Few right-hand sides: at most 4 run as one pass over the digit planes
    (one wave per row, 1 KB blocks of k, a 256-byte tail at 40 x 33), more as
    one padded 128-column tile with k split over several workgroups.  Forward
    and adjoint bit for bit against the oracle's integer product."""
    announce(f"int8 few rhs nx={nx} ny={ny} nrhs={nrhs} bits={bits} rho_bits={rho_bits}")
    g = np.random.default_rng(nx * nrhs + bits)
    ub = g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g), ub)
    N = G.shape[0]
    rho = g.uniform(-1, 1, (nrhs, N))
    if nrhs > 1:
        rho[1] = 0.0
    ref, _, _ = oracle_int8(G, bits // 8, rho.T, rho_bits // 8, h, w)
    S, Sg = bits // 8, rho_bits // 8
    qG, e = quant.quantize_rows(G, S)
    qg, f = quant.quantize_cols(rho.T, Sg, pre_exponent=e)
    ref_adj, _ = apply.integer_apply(qG.T, e, S, qg, f, Sg, h, None, row_exponent=False)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.quantize(bits)
        u = host(op.apply(dev(rho), "int8", rho_bits))
        lam = host(op.apply_adjoint(dev(rho), "int8", rho_bits))
    assert np.array_equal(u.T, ref)
    assert np.array_equal(lam.T, ref_adj)


@pytest.mark.parametrize("nx,ny", [(12, 9), (50, 37), (66, 66)])
def test_int8_adjoint_bit_exact(torch, pinv, nx, ny):
    """(66, 66): P = 4096 with one tile column, so the product splits k."""
    announce(f"adjoint int8 nx={nx} ny={ny}")
    g = np.random.default_rng(11)
    h = 1.0 / (max(nx, ny) - 1)
    G, _, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g))
    N = G.shape[0]
    gv = g.standard_normal((70, N))
    S, Sg = 2, 2
    qG, e = quant.quantize_rows(G, S)
    qg, f = quant.quantize_cols(gv.T, Sg, pre_exponent=e)
    ref, _ = apply.integer_apply(qG.T, e, S, qg, f, Sg, h, None, row_exponent=False)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.quantize(16)
        lam = host(op.apply_adjoint(dev(gv), "int8", 16))
    assert np.array_equal(lam.T, ref)


# ---------------------------------------------------------------- split precision

@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("nx,ny", [(12, 9), (66, 66)])
def test_split_modes_against_emulation(torch, pinv, mode, nx, ny):
    """The GPU differs from the exact-product emulation only by FP32
    accumulation (element by element), stays inside the operand-rounding
    envelope of the FP64 solve, and FP32 / BF16x6 are separated from BF16x3
    (check_split_solve).  (66, 66) runs several tiles and split k."""
    announce(f"apply {mode} nx={nx} ny={ny}")
    g = np.random.default_rng(5)
    h = 1.0 / (max(nx, ny) - 1)
    G, _, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g))
    rho = g.uniform(-1, 1, (40, G.shape[0]))
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.prepare_split(mode)
        u = host(op.apply(dev(rho), mode))
    err = check_split_solve(u.T, G, rho.T, h, mode)
    print(f"[split {nx}x{ny}] {mode}: max rel L2 vs FP64 {err.max():.3e}", flush=True)


@pytest.mark.parametrize("nrhs", [1000, 1100])
def test_bf16x3_on_wide_tiles(torch, pinv, nrhs):
    """BF16x3 with at least 128 tiles of 128 x 256 runs the one-wave-per-SIMD
    kernel: 4096 unknowns x 1000 right-hand sides is 32 x 4 tiles with k split
    in two (ragged last column tile), x 1100 is 32 x 5 tiles without a split.
    Element by element against the exact-product emulation, and within the
    operand-rounding envelope of the FP64 solve (check_split_solve)."""
    nx = ny = 66
    announce(f"apply bf16x3 on 128 x 256 tiles nx={nx} nrhs={nrhs}")
    g = np.random.default_rng(nrhs)
    h = 1.0 / (nx - 1)
    ub = g.standard_normal((ny, nx))
    G, w, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g), ub)
    rho = g.uniform(-1, 1, (nrhs, G.shape[0]))
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.prepare_split("bf16x3")
        u = host(op.apply(dev(rho), "bf16x3"))
    # the lift is added exactly in FP64 after the product
    u = u - w[None, :]
    err = check_split_solve(u.T, G, rho.T, h, "bf16x3")
    print(f"[bf16x3 wide] nrhs={nrhs}: max rel L2 vs FP64 {err.max():.3e}", flush=True)


# ---------------------------------------------------------------- derivatives

@pytest.mark.parametrize("nx,ny,R", [(12, 9, 6), (40, 33, 6), (40, 33, 53), (17, 23, 16)])
def test_fp64_adjoint_and_grad_eps(torch, pinv, nx, ny, R):
    """R > 16 runs the chunked two-kernel path (53 = three full chunks and a
    ragged one); R <= 16 the single-kernel path."""
    announce(f"adjoint fp64 + grad_eps nx={nx} ny={ny} nrhs={R}")
    g = np.random.default_rng(21)
    h = 1.0 / (max(nx, ny) - 1)
    eps = workloads.random_eps(nx, ny, g)
    ub = g.standard_normal((ny, nx))
    G, w, _ = oracle_inverse(nx, ny, eps, ub)
    N = G.shape[0]
    rho = g.standard_normal((R, N))
    gv = g.standard_normal((R, N))
    u_ref = apply.plain_apply(G, rho.T, h, w)
    lam_ref = grad.adjoint(G, gv.T, h)
    ge_ref = grad.grad_eps_nodes(nx, ny, h, u_ref, lam_ref, ub)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, eps, ub, w) as op:
        u = op.apply(dev(rho), "fp64")
        lam = op.apply_adjoint(dev(gv), "fp64")
        ge = host(op.grad_eps(u, lam))
        lam = host(lam)
    assert np.max(metrics.rel_l2_per_rhs(lam.T, lam_ref)) <= 1e-12
    assert np.linalg.norm(ge - ge_ref) <= 1e-12 * np.linalg.norm(ge_ref)


@pytest.mark.parametrize("R", [3, 40])
def test_fp64_adjoint_of_exactly_symmetric_and_other_inverses(torch, pinv, R):
    """The FP64 adjoint runs the forward product when G equals G^T bit for bit
    (checked when G is built, imported or loaded): a GPU-built operator, an
    imported symmetrised inverse; and the transposed product otherwise (an
    imported inverse with one entry pair made unequal).  Each against the
    oracle's G^T product, and the symmetric ones bit for bit against the
    forward apply of the same vectors.  R = 3: GEMV; 40: the tiled product."""
    nx, ny = 40, 33
    announce(f"fp64 adjoint, symmetric shortcut nrhs={R}")
    g = np.random.default_rng(5 + R)
    h = 1.0 / (nx - 1)
    eps = workloads.random_eps(nx, ny, g)
    G, _, _ = oracle_inverse(nx, ny, eps)
    N = G.shape[0]
    gv = g.standard_normal((R, N))
    Gs = 0.5 * (G + G.T)                  # exactly symmetric
    Gn = Gs.copy()
    Gn[3, 17] *= 1.0 + 1e-9               # not symmetric
    with pinv.PoissonInverse.build(nx, ny, h, eps) as op:
        assert op.info()["fp64_symmetric"] == 1
        Gb, _ = op.export_inverse()
        assert np.array_equal(Gb, Gb.T)
        lam = op.apply_adjoint(dev(gv), "fp64")
        assert torch.equal(lam, op.apply(dev(gv), "fp64"))
        assert np.max(metrics.rel_l2_per_rhs(host(lam).T, grad.adjoint(Gb, gv.T, h))) <= 1e-12
    for M, sym in ((Gs, 1), (Gn, 0)):
        with pinv.PoissonInverse.from_inverse(nx, ny, h, M) as op:
            assert op.info()["fp64_symmetric"] == sym
            lam = op.apply_adjoint(dev(gv), "fp64")
            if sym:
                assert torch.equal(lam, op.apply(dev(gv), "fp64"))
            assert np.max(metrics.rel_l2_per_rhs(host(lam).T, grad.adjoint(M, gv.T, h))) <= 1e-12


def test_grad_eps_without_right_hand_sides_is_zero(torch, pinv):
    announce("grad_eps nrhs=0")
    nx, ny = 10, 8
    G, _, _ = oracle_inverse(nx, ny)
    with pinv.PoissonInverse.from_inverse(nx, ny, 0.1, G) as op:
        empty = torch.empty((0, op.n), dtype=torch.float64, device="cuda")
        out = torch.full((ny, nx), float("nan"), dtype=torch.float64, device="cuda")
        op.grad_eps(empty, empty, out=out)
        assert float(out.abs().sum()) == 0.0


def test_autograd_matches_finite_differences(torch, pinv):
    """Gradients of sum_r ||C u_r - d_r||^2 through PinvSolve (GPU build, FP64
    mode) against central differences of fresh FP64 banded solves."""
    from paper_1602_00001_amd.autograd import PinvSolve
    announce("autograd PinvSolve vs central differences nx=24 ny=20")
    g = np.random.default_rng(8)
    nx, ny = 24, 20
    h = 1.0 / (nx - 1)
    N = (nx - 2) * (ny - 2)
    eps = 1.0 + 0.5 * g.uniform(0, 1, (ny, nx))
    rho = g.standard_normal((4, N))
    sample = np.sort(g.choice(N, 30, replace=False))
    d = 0.01 * g.standard_normal((30, 4))
    with pinv.PoissonInverse.build(nx, ny, h, eps) as op:
        rt = dev(rho).requires_grad_(True)
        et = dev(eps).requires_grad_(True)
        u = PinvSolve.apply(rt, et, op, "fp64", 16)
        idx = torch.from_numpy(sample).cuda()
        loss = ((u[:, idx] - dev(d.T)) ** 2).sum()
        loss.backward()
        ge = host(et.grad)
        gr = host(rt.grad)

    def lossf(e):
        return grad.sampling_loss(nx, ny, h, e, rho.T, sample, d)

    for t in range(3):
        v = g.standard_normal((ny, nx))
        fd = grad.central_difference(lossf, eps, v, 1e-6)
        assert abs(fd - float(np.sum(ge * v))) <= 1e-6 * abs(fd)
    v = g.standard_normal(rho.shape)
    fd = grad.central_difference(lambda r: grad.sampling_loss(nx, ny, h, eps, r.T, sample, d), rho, v, 1e-6)
    assert abs(fd - float(np.sum(gr * v))) <= 1e-6 * abs(fd)


# ---------------------------------------------------------------- argument checks on the device path

def test_invalid_arguments(torch, pinv):
    announce("invalid arguments")
    nx, ny, h = 10, 10, 0.1
    G, _, _ = oracle_inverse(nx, ny)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        x = dev(np.ones((2, G.shape[0])))
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(x, "int8", 16)
        assert ei.value.status == pinv.E_STATE
        op.quantize(16)
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(x, "int8", 12)
        assert ei.value.status == pinv.E_INVALID_ARG
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(x, "fp64", out=x)          # overlapping input and output
        assert ei.value.status == pinv.E_INVALID_ARG
        with pytest.raises(pinv.PinvError) as ei:
            op.quantize(12)
        assert ei.value.status == pinv.E_INVALID_ARG
        op.quantize(16, keep_fp64=False)
        with pytest.raises(pinv.PinvError) as ei:
            op.apply(x, "fp64")
        assert ei.value.status == pinv.E_STATE
        assert op.apply(x, "int8", 16).shape == x.shape


def test_int8_apply_long_columns_bit_exact(torch, pinv):
    """Right-hand sides of 16500 entries take the 1024-thread quantiser (columns
    of 16385-40960 entries held in registers): bit for bit against the oracle's
    integer apply, on an imported random inverse."""
    nx, ny = 1652, 12                       # N = 1650 * 10 = 16500
    N = (nx - 2) * (ny - 2)
    announce(f"int8 apply, long columns N={N}")
    g = np.random.default_rng(23)
    G = g.standard_normal((N, N))
    rho = g.uniform(-1, 1, (3, N))
    rho[1] *= 1e-5
    h = 0.01
    ref, _, _ = oracle_int8(G, 3, rho.T, 2, h)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        del G
        op.quantize(24, keep_fp64=False)
        u = host(op.apply(dev(rho), "int8", 16))
    assert np.array_equal(u.T, ref)
