"""Time-coupled stepping (one right-hand side per step, each depending on the
previous solution): rho_{t+1} = rho_t + tau * u_t on the 32x32 grid, 64 steps.
The GPU loop (FP64 GEMV apply + the coupling update) against the same loop run
by the oracle's plain apply in FP64; the loop captured once in a HIP graph and
replayed against the eager loop, bit for bit."""

import numpy as np
import pytest

from oracle import apply, grid, inverse
from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_coupled_32_against_oracle_and_graph(torch):
    from paper_1602_00001_amd import pinv
    wl = workloads.coupled_32()
    n, h, tau, steps = wl["n"], wl["h"], wl["tau"], wl["steps"]
    announce(f"coupled_32: {steps} coupled steps, tau={tau}")
    K, _ = grid.conservative_operator(n, n, None)
    G = inverse.lu_inverse(K)
    rho = wl["rho0"].T.copy()                                 # [N, 1]
    for _ in range(steps):
        u = apply.plain_apply(G, rho, h, None)
        rho = rho + tau * u
    ref_rho, ref_u = rho, u

    with pinv.PoissonInverse.build(n, n, h) as op:
        r = dev(wl["rho0"])
        u_t = torch.empty_like(r)

        def loop():
            for _ in range(steps):
                op.apply(r, "fp64", out=u_t)
                r.add_(u_t, alpha=tau)

        loop()
        eager_rho, eager_u = r.clone(), u_t.clone()
        scale = np.max(np.abs(ref_rho))
        assert np.max(np.abs(host(eager_rho).T - ref_rho)) <= 1e-11 * scale
        assert np.max(np.abs(host(eager_u).T - ref_u)) <= 1e-11 * np.max(np.abs(ref_u))

        announce("coupled_32: HIP graph of the loop")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            r.copy_(dev(wl["rho0"]))
            op.apply(r, "fp64", out=u_t)
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            loop()
        for rep in range(3):
            r.copy_(dev(wl["rho0"]))
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(r, eager_rho) and torch.equal(u_t, eager_u), rep
        del graph
