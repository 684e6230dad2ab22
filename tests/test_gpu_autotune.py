"""Int8 kernel variants: every variant gives the oracle's integer result bit for
bit (forward and adjoint, several slice counts, a grid whose tile count is not a
multiple of eight), and autotuning picks a valid variant, reports a time for
each, and leaves the results unchanged."""

import numpy as np
import pytest

from oracle import apply, quant
from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, dev, host, oracle_inverse, oracle_int8, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


@pytest.mark.parametrize("nx,ny,bits,rho_bits", [(40, 31, 24, 16), (33, 20, 16, 24), (12, 9, 8, 8), (66, 66, 24, 16),
                                                 (14, 14, 24, 16), (19, 19, 16, 16), (22, 22, 8, 16)])
def test_every_variant_bit_exact(torch, pinv, nx, ny, bits, rho_bits):
    """(66, 66) has P = 4096 and few tiles, so every variant also runs split
    over k (integer class sums of the splits added exactly).  The k loops run
    1 to 32 steps of 128 bytes; (14, 14), (19, 19) and (22, 22) give 2, 3 and
    4 steps, where the one-wave-per-SIMD schedule has no step, one step or two
    steps that load a stage two ahead."""
    g = np.random.default_rng(nx * ny + bits)
    ub = g.standard_normal((ny, nx))
    h = 1.0 / (max(nx, ny) - 1)
    G, w, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g), ub)
    N = G.shape[0]
    rho = g.uniform(-1, 1, (300, N))
    ref, _, _ = oracle_int8(G, bits // 8, rho.T, rho_bits // 8, h, w)
    gv = g.standard_normal((70, N))
    S, Sg = bits // 8, rho_bits // 8
    qG, e = quant.quantize_rows(G, S)
    qg, f = quant.quantize_cols(gv.T, Sg, pre_exponent=e)
    ref_adj, _ = apply.integer_apply(qG.T, e, S, qg, f, Sg, h, None, row_exponent=False)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.quantize(bits)
        for v in range(pinv.int8_variants()):
            announce(f"int8 variant {v} nx={nx} ny={ny} bits={bits} rho_bits={rho_bits}")
            op.set_int8_variant(rho_bits, v)
            u = host(op.apply(dev(rho), "int8", rho_bits))
            assert np.array_equal(u.T, ref), v
            lam = host(op.apply_adjoint(dev(gv), "int8", rho_bits))
            assert np.array_equal(lam.T, ref_adj), v


def test_autotune_picks_a_variant_and_keeps_results(torch, pinv):
    nx = ny = 50
    g = np.random.default_rng(77)
    h = 1.0 / (nx - 1)
    G, _, _ = oracle_inverse(nx, ny)
    rho = g.uniform(-1, 1, (200, G.shape[0]))
    ref, _, _ = oracle_int8(G, 3, rho.T, 2, h)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        with pytest.raises(pinv.PinvError) as ei:
            op.autotune_int8(16, nrhs=256, reps=2)
        assert ei.value.status == pinv.E_STATE
        op.quantize(24)
        for src in ("random digits", "caller rho"):
            announce(f"autotune int8 50x50 on {src}, 3 reps")
            if src == "caller rho":
                best, ms = op.autotune_int8(16, rho=dev(rho), reps=3)
            else:
                best, ms = op.autotune_int8(16, nrhs=256, reps=3)
            print(f"[autotune] {src}: best {best} ms {ms}", flush=True)
            assert 0 <= best < pinv.int8_variants()
            assert len(ms) == pinv.int8_variants() and all(t > 0 for t in ms)
            assert ms[best] == min(ms)
            u = host(op.apply(dev(rho), "int8", 16))
            assert np.array_equal(u.T, ref)
        for bad in [dict(nrhs=0), dict(nrhs=10, reps=0), dict(rho_bits=12, nrhs=10)]:
            kw = dict(rho_bits=16, reps=1)
            kw.update(bad)
            with pytest.raises(pinv.PinvError) as ei:
                op.autotune_int8(**kw)
            assert ei.value.status == pinv.E_INVALID_ARG
        with pytest.raises(pinv.PinvError):
            op.set_int8_variant(16, pinv.int8_variants())


def test_split_of_the_last_round_of_tiles(torch, pinv):
    """4096 unknowns x 1100 right-hand sides: 288 tiles of 128 x 128 for 256
    resident workgroups (576 of 64 x 128 for 512), so the last round's row
    tiles run split over k and the rest unsplit.  Every variant gives the
    allocation-free apply's result (which never splits k) bit for bit, and
    sampled columns of it and of the adjoint the oracle's integer result."""
    nx = ny = 66
    g = np.random.default_rng(5)
    h = 1.0 / (nx - 1)
    ub = g.standard_normal((ny, nx))
    G, w, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g), ub)
    N = G.shape[0]
    R = 1100
    rho = g.uniform(-1, 1, (R, N))
    gv = g.uniform(-1, 1, (R, N))
    cols = np.sort(g.choice(R, 8, replace=False))
    ref, _, _ = oracle_int8(G, 3, rho[cols].T, 2, h, w)
    qG, e = quant.quantize_rows(G, 3)
    qg, f = quant.quantize_cols(gv[cols].T, 2, pre_exponent=e)
    ref_adj, _ = apply.integer_apply(qG.T, e, 3, qg, f, 2, h, None, row_exponent=False)
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G, None, ub, w) as op:
        op.quantize(24)
        x, xg = dev(rho), dev(gv)
        announce("int8 4096 x 1100, unsplit reference (allocation-free apply)")
        unsplit = host(op.apply_noalloc(x, 16))
        assert np.array_equal(unsplit[cols].T, ref)
        for v in range(pinv.int8_variants()):
            announce(f"int8 variant {v}, 4096 x 1100 (last round split over k)")
            op.set_int8_variant(16, v)
            u = host(op.apply(x, "int8", 16))
            assert np.array_equal(u, unsplit), v
            lam = host(op.apply_adjoint(xg, "int8", 16))
            assert np.array_equal(lam[cols].T, ref_adj), v


def test_autotune_cache_file(torch, pinv, tmp_path, monkeypatch):
    """PINV_AUTOTUNE_CACHE: the first tuning appends its choice; a second op
    of the same size takes it from the file without timing (the others'
    times reported as -1); another right-hand-side count is tuned afresh;
    results stay the oracle's."""
    nx = ny = 40
    g = np.random.default_rng(9)
    h = 1.0 / (nx - 1)
    G, _, _ = oracle_inverse(nx, ny)
    rho = g.uniform(-1, 1, (150, G.shape[0]))
    ref, _, _ = oracle_int8(G, 2, rho.T, 2, h)
    cache = tmp_path / "tune.txt"
    cache.write_text("a line that is not an entry\nint8 short\n")
    monkeypatch.setenv("PINV_AUTOTUNE_CACHE", str(cache))
    nv = pinv.int8_variants()
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.quantize(16)
        announce("autotune with an empty cache file")
        best, ms = op.autotune_int8(16, nrhs=150, reps=2)
        assert all(t > 0 for t in ms) and ms[best] == min(ms)
        lines = cache.read_text().splitlines()
        entry = lines[-1].split()
        assert len(lines) == 3 and entry[0] == "int8" and entry[3:8] == [str(G.shape[0]), "2", "2", "256", str(best)]
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        op.quantize(16)
        announce("autotune served from the cache file")
        best2, ms2 = op.autotune_int8(16, nrhs=150, reps=2)
        assert best2 == best
        assert ms2[best] > 0 and all(t == -1.0 for v, t in enumerate(ms2) if v != best)
        assert len(cache.read_text().splitlines()) == 3
        u = host(op.apply(dev(rho), "int8", 16))
        assert np.array_equal(u.T, ref)
        announce("autotune for another right-hand-side count")
        _, ms3 = op.autotune_int8(16, nrhs=300, reps=1)
        assert all(t > 0 for t in ms3)
        assert len(cache.read_text().splitlines()) == 4
    assert nv == len(ms)
