"""Shared helpers of the GPU parity tests (test infrastructure)."""

import numpy as np
import pytest

from oracle import apply, grid, inverse, quant


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1602_00001_amd import pinv  # noqa: F401  (fails loudly without the library)
    return torch


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_inverse(nx, ny, eps=None, ub=None):
    """(G, w, bB) from the oracle: conservative operator and its LU inverse."""
    K, bB = grid.conservative_operator(nx, ny, eps, ub)
    G = inverse.lu_inverse(K)
    w = apply.lift(G, bB) if ub is not None else None
    return G, w, bB


def oracle_int8(G, S, rho_cols, Sr, h, w=None):
    """Oracle quantised solve; rho_cols is [N, R]."""
    qG, e = quant.quantize_rows(G, S)
    qR, f = quant.quantize_cols(rho_cols, Sr)
    u, acc = apply.integer_apply(qG, e, S, qR, f, Sr, h, w)
    return u, qG, e


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
