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


def split_tolerances(G, rho_cols, mode):
    """Per-RHS bounds for a split-precision solve, derived from the arithmetic.

    kappa_r = || |G| |rho_r| || / || G rho_r || measures cancellation in the
    product.  Operand rounding: unit roundoff u_op (2^-24 for FP32; the
    neglected parts of a bfloat16 split are below 2^-16 for 2 parts and 2^-24
    for 3 parts, relative to each operand) gives |error| <= 2 u_op kappa.
    FP32 accumulation over N terms adds at most ~sqrt(N) 2^-24 kappa
    (statistical bound, with a factor 4 of slack).
    Returns (bound vs FP64, bound vs the exact-product emulation), arrays [R].
    """
    A = np.abs(G) @ np.abs(rho_cols)
    U = G @ rho_cols
    kappa = np.linalg.norm(A, axis=0) / np.maximum(np.linalg.norm(U, axis=0), 1e-300)
    u_op = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "bf16x6": 2.0 ** -24}[mode]
    acc = 4.0 * np.sqrt(G.shape[0]) * 2.0 ** -24 * kappa
    return 2.0 * u_op * kappa + acc, acc
