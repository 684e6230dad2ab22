"""Applies captured in a HIP graph: the FP64 GEMV apply (at most 4 right-hand
sides; allocates nothing), the FP64 GEMM apply (packing kernel, stream-ordered
scratch; split k at 64^2), the int8 apply (its stream-ordered scratch becomes
alloc and free nodes; the split-K epilogue at 64^2) and the symmetric-packed
FP64 apply.  Every replay, with eager work and synchronisations in between,
gives the eager result bit for bit."""

import numpy as np
import pytest

from oracle import apply
from tests.gpu_util import announce, dev, host, oracle_inverse, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("nrhs", [1, 3])
def test_graph_replay_of_fp64_gemv_apply(torch, nrhs):
    from paper_1602_00001_amd import pinv
    announce(f"HIP graph of 8 fp64 GEMV applies, nrhs={nrhs}")
    nx, ny = 32, 32
    h = 1.0 / (nx - 1)
    G, _, _ = oracle_inverse(nx, ny)
    g = np.random.default_rng(60 + nrhs)
    rho_h = g.standard_normal((nrhs, G.shape[0]))
    with pinv.PoissonInverse.from_inverse(nx, ny, h, G) as op:
        rho = dev(rho_h)
        eager = op.apply(rho, "fp64")
        u = torch.full_like(rho, float("nan"))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            op.apply(rho, "fp64", out=u)
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(8):
                op.apply(rho, "fp64", out=u)
        ref = apply.plain_apply(G, rho_h.T, h, None)
        for rep in range(4):
            u.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(u, eager), rep
            # eager work between replays
            other = op.apply(dev(g.standard_normal((nrhs, G.shape[0]))), "fp64")
            torch.cuda.synchronize()
            del other
        assert np.max(np.abs(host(u).T - ref)) <= 1e-12 * np.max(np.abs(ref))
        del graph


@pytest.mark.parametrize("nx,nrhs,mode", [(32, 200, "int8"), (66, 200, "int8"), (40, 3, "fp64_sym"),
                                          (40, 5, "fix16_tile"), (32, 200, "fp64"), (66, 200, "fp64")])
def test_graph_replay_of_int8_and_packed_applies(torch, nx, nrhs, mode):
    from paper_1602_00001_amd import pinv
    announce(f"HIP graph of 4 {mode} applies nx={nx} nrhs={nrhs}")
    h = 1.0 / (nx - 1)
    G, _, _ = oracle_inverse(nx, nx)
    g = np.random.default_rng(nx + nrhs)
    with pinv.PoissonInverse.from_inverse(nx, nx, h, G) as op:
        if mode == "int8":
            op.quantize(24)
        elif mode != "fp64":
            op.prepare_split(mode)
        rho = dev(g.uniform(-1, 1, (nrhs, G.shape[0])))
        eager = op.apply(rho, mode, 16)
        u = torch.full_like(rho, float("nan"))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            op.apply(rho, mode, 16, out=u)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(4):
                op.apply(rho, mode, 16, out=u)
        for rep in range(4):
            u.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(u, eager), rep
            other = op.apply(dev(g.uniform(-1, 1, (nrhs, G.shape[0]))), mode, 16)
            torch.cuda.synchronize()
            del other
        if mode == "fp64":
            ref = apply.plain_apply(G, host(rho).T, h, None)
            assert np.max(np.abs(host(u).T - ref)) <= 1e-12 * np.max(np.abs(ref))
        del graph
