"""A 258 x 258 grid, N = 256^2 = 65536 interior unknowns, a 34 GB FP64
inverse built on the GPU.  FP64 applies against the oracle's banded-Cholesky
solve; 8-bit entries x 16-bit right-hand sides within their envelope; 24-bit
entries x 16-bit right-hand sides, where two digit pairs share a class and
N * 128 * 128 * 2 reaches 2^31, run with k split (int32 class sums per part,
added in int64) within their envelope; the grouped batched product, which does
not split k, refuses that op."""

import numpy as np
import pytest

from oracle import grad, metrics
from paper_1602_00001_amd import workloads
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def test_max_size_operator():
    torch = require_gpu()
    from paper_1602_00001_amd import pinv
    n = 258
    h = 1.0 / (n - 1)
    N = (n - 2) ** 2
    announce(f"max size: {n}x{n} grid, N = {N}, FP64 inverse {8 * N * N / 1e9:.1f} GB")
    rho = workloads.blob_rhs(n, 6, workloads.rng(9, 0))
    ref = grad.banded_solve(n, n, h, np.ones((n, n)), rho.T)
    with pinv.PoissonInverse.build(n, n, h) as op:
        assert op.n == N
        u = host(op.apply(dev(rho), "fp64"))
        err = np.max(metrics.rel_l2_per_rhs(u.T, ref))
        print(f"[max size] fp64 vs banded solve: {err:.3e}", flush=True)
        assert err <= 1e-10
        op.quantize(8)
        u8 = host(op.apply(dev(rho), "int8", 16))
        err8 = np.max(metrics.rel_l2_per_rhs(u8.T, u.T))
        print(f"[max size] 8-bit x 16-bit vs fp64: {err8:.3e}", flush=True)
        assert err8 <= 2.0 ** -6
        op.quantize(24)
        u24 = host(op.apply(dev(rho), "int8", 16))
        err24 = np.max(metrics.rel_l2_per_rhs(u24.T, u.T))
        print(f"[max size] 24-bit x 16-bit (k split) vs fp64: {err24:.3e}", flush=True)
        assert err24 <= 2.0 ** -14
        x = dev(rho)
        with pytest.raises(pinv.PinvError) as ei:
            pinv.apply_batched([(op, x, torch.empty_like(x))], "int8", 16)
        assert ei.value.status == pinv.E_UNSUPPORTED
