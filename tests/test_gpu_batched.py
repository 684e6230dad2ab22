"""Batched uneven requests: pinv_apply_batched equals one pinv_apply_inverse per
request, bit for bit in INT8 mode (the grouping only changes which columns share
a launch; every column's quantisation and integer product are independent),
and the per-request results match the oracle.  The operators carry different
inverse precisions (one grouped launch per digit count, its kernel variant
timed on it when the request list is first planned).  A request list's plan is cached: a captured HIP graph of
the call replays bit-identically, and re-quantising an op drops its plans."""

import numpy as np
import pytest

from oracle import apply, quant
from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, dev, host, oracle_inverse, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pinv():
    from paper_1602_00001_amd import pinv as p
    return p


GRIDS = [(12, 9), (20, 20), (33, 17), (40, 40), (25, 30)]
BITS = [16, 24, 8, 16, 24]
VARIANTS = [None, 3, None, 8, 13]   # per-op variants (single applies); batched launches time their own


@pytest.fixture(scope="module")
def ops(torch, pinv):
    g = np.random.default_rng(40)
    out = []
    for (nx, ny), bits, var in zip(GRIDS, BITS, VARIANTS):
        eps = workloads.random_eps(nx, ny, g)
        ub = g.standard_normal((ny, nx)) if nx == 20 else None
        h = 1.0 / (max(nx, ny) - 1)
        G, w, _ = oracle_inverse(nx, ny, eps, ub)
        op = pinv.PoissonInverse.from_inverse(nx, ny, h, G, eps, ub, w)
        op.quantize(bits)
        if var is not None:
            for rb in (8, 16, 24):
                op.set_int8_variant(rb, var)
        out.append(dict(op=op, G=G, w=w, h=h, S=bits // 8))
    yield out
    for o in out:
        o["op"].close()


def _requests(torch, ops, seed, nreq=40):
    g = np.random.default_rng(seed)
    reqs = []
    for _ in range(nreq):
        k = int(g.integers(0, len(ops)))
        n = ops[k]["op"].n
        nrhs = int(g.integers(0, 71))
        pad = int(g.integers(0, 5))
        rho_h = g.uniform(-1, 1, (nrhs, n + pad))
        rho = dev(rho_h)[:, :n]
        u = torch.full((nrhs, n + pad), float("nan"), dtype=torch.float64, device="cuda")[:, :n]
        reqs.append((k, rho, u, rho_h[:, :n]))
    return reqs


@pytest.mark.parametrize("rho_bits", [8, 16, 24])
def test_batched_int8_equals_per_request(torch, pinv, ops, rho_bits):
    announce(f"apply_batched int8 rho_bits={rho_bits} 60 requests over {len(GRIDS)} ops")
    reqs = _requests(torch, ops, 100 + rho_bits, 60)
    pinv.apply_batched([(ops[k]["op"], rho, u) for (k, rho, u, _) in reqs], "int8", rho_bits)
    for (k, rho, u, rho_h) in reqs:
        if rho.shape[0] == 0:
            continue
        single = host(ops[k]["op"].apply(rho, "int8", rho_bits))
        assert np.array_equal(host(u), single)
    # and one request per operator against the oracle
    for k, o in enumerate(ops):
        mine = [r for r in reqs if r[0] == k and r[1].shape[0] > 0]
        if not mine:
            continue
        _, _, u, rho_h = mine[0]
        qG, e = quant.quantize_rows(o["G"], o["S"])
        qR, f = quant.quantize_cols(rho_h.T, rho_bits // 8)
        ref, _ = apply.integer_apply(qG, e, o["S"], qR, f, rho_bits // 8, o["h"], o["w"])
        assert np.array_equal(host(u).T, ref)


def test_batched_fp64_equals_per_request(torch, pinv, ops):
    announce("apply_batched fp64 40 requests")
    reqs = _requests(torch, ops, 7)
    pinv.apply_batched([(ops[k]["op"], rho, u) for (k, rho, u, _) in reqs], "fp64")
    for (k, rho, u, rho_h) in reqs:
        if rho.shape[0] == 0:
            continue
        assert np.array_equal(host(u), host(ops[k]["op"].apply(rho, "fp64")))


def test_batched_rejects_unquantised_op(torch, pinv):
    announce("apply_batched with an unquantised op -> E_STATE, nothing launched")
    nx = ny = 10
    G, _, _ = oracle_inverse(nx, ny)
    with pinv.PoissonInverse.from_inverse(nx, ny, 0.1, G) as op:
        rho = dev(np.ones((2, op.n)))
        u = torch.zeros_like(rho)
        with pytest.raises(pinv.PinvError) as ei:
            pinv.apply_batched([(op, rho, u)], "int8", 16)
        assert ei.value.status == pinv.E_STATE
        assert float(u.abs().sum()) == 0.0


def _capture_list(torch, ops, seed, nreq=24):
    reqs = _requests(torch, ops, seed, nreq)
    return reqs, [(ops[k]["op"], rho, u) for (k, rho, u, _) in reqs]


def test_batched_graph_capture_replays_bit_identical(torch, pinv, ops):
    """A request list planned by an eager call on a stream, then captured on
    that stream into a HIP graph: every replay (with other batched and single
    applies in between) reproduces the eager result bit for bit."""
    announce("apply_batched int8 graph capture: eager plan, capture, 3 replays")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    reqs, batch = _capture_list(torch, ops, 321)
    with torch.cuda.stream(s):
        pinv.apply_batched(batch, "int8", 16, stream=s)
    s.synchronize()
    eager = [host(u).copy() for (_, _, u) in batch]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pinv.apply_batched(batch, "int8", 16, stream=s)
    other_reqs, other = _capture_list(torch, ops, 654)
    for rep in range(3):
        for (_, _, u) in batch:
            u.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, (_, _, u) in zip(eager, batch):
            assert np.array_equal(host(u), e), rep
        # eager work between replays: another request list, a single apply
        pinv.apply_batched(other, "int8", 16)
        k, rho, u, _ = other_reqs[0]
        ops[k]["op"].apply(rho, "int8", 16, out=u)
        torch.cuda.synchronize()
    del g


def test_batched_plans_follow_requantisation(torch, pinv):
    """A plan names its ops' digit planes: re-quantising an op (new planes,
    another digit count) drops it, and the next call with the same requests
    uses the new planes (bit-identical to per-request applies)."""
    g = np.random.default_rng(77)
    nx = ny = 30
    G, _, _ = oracle_inverse(nx, ny, workloads.random_eps(nx, ny, g))
    with pinv.PoissonInverse.from_inverse(nx, ny, 1.0 / (nx - 1), G) as op:
        rho = dev(g.uniform(-1, 1, (50, op.n)))
        u, u2 = torch.empty_like(rho), torch.empty_like(rho[:7])
        for bits in (16, 24, 16):
            announce(f"apply_batched after quantize({bits})")
            op.quantize(bits)
            pinv.apply_batched([(op, rho, u), (op, rho[:7], u2)], "int8", 16)
            assert np.array_equal(host(u), host(op.apply(rho, "int8", 16)))
            assert np.array_equal(host(u2), host(op.apply(rho[:7], "int8", 16)))
    pinv.batched_release()
