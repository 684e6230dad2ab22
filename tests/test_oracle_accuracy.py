"""The accuracy contract of the quantised solve: with b-bit per-row entries and
a right-hand side rounded to at least b bits (16 at least), the relative L2
error against the FP64 solve stays within 2^-(b-2) on smooth right-hand sides
(Gaussian blobs, variable eps), b = 8, 16, 24.  (On iid uniform right-hand
sides per-row 16-bit entries miss it, which is why the metric's workload uses
24-bit entries.)"""

import numpy as np
import pytest

from oracle import apply, grid, inverse, metrics, quant
from paper_1602_00001_amd import workloads


@pytest.mark.parametrize("n", [32, 48])
@pytest.mark.parametrize("bits", [8, 16, 24])
def test_quantised_solve_within_envelope(n, bits):
    h = 1.0 / (n - 1)
    K, _ = grid.conservative_operator(n, n, workloads.eps_sincos(n))
    G = inverse.lu_inverse(K)
    rho = workloads.blob_rhs(n, 12, workloads.rng(7, n)).T
    ref = apply.plain_apply(G, rho, h)
    S, Sr = bits // 8, max(bits, 16) // 8
    qG, e = quant.quantize_rows(G, S)
    qR, f = quant.quantize_cols(rho, Sr)
    u, _ = apply.integer_apply(qG, e, S, qR, f, Sr, h)
    err = np.max(metrics.rel_l2_per_rhs(u, ref))
    assert err <= 2.0 ** -(bits - 2), err
    # and it is a real rounding error, not a loss of the solution
    assert err > 2.0 ** -(bits + 10)
