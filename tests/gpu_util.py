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


def rounding_model(G, rho_cols, S, Sr):
    """Statistical size of the quantised solve's relative L2 error, per
    right-hand side, from the arithmetic of the per-row rounding.

    Rounding G_ik to q_ik 2^e_i / M_S errs by at most 2^e_i / (2 M_S); taken
    as independent and uniform, the errors have variance 4^e_i / (12 M_S^2),
    so E ||dG rho_r||^2 = sum_i 4^e_i / (12 M_S^2) ||rho_r||^2.  Rounding rho_r
    with its column exponent f_r adds E ||G drho_r||^2 = 4^f_r / (12 M_Sr^2)
    ||G||_F^2.  Returns (G part, rho part), each divided by ||G rho_r|| (the
    factor h^2 cancels); their root sum of squares is the expected error.
    kappa_q = (G part) / 2^-(b-2) is the factor by which the data amplify the
    2^-(b-2) contract: below 1 for smooth positive right-hand sides, about 3
    for iid uniform ones (mean zero: G rho cancels)."""
    e = quant.frexp_exponent(np.max(np.abs(G), axis=1))
    f = quant.frexp_exponent(np.max(np.abs(rho_cols), axis=0))
    M, Mr = float(quant.max_mag(S)), float(quant.max_mag(Sr))
    den = np.linalg.norm(G @ rho_cols, axis=0)
    vG = np.sum(4.0 ** e) / (12.0 * M * M) * np.sum(rho_cols ** 2, axis=0)
    vR = 4.0 ** f / (12.0 * Mr * Mr) * np.sum(G ** 2)
    return np.sqrt(vG) / den, np.sqrt(vR) / den


def split_term_magnitudes(G, rho_cols, mode):
    """T[i, r]: the sum of the magnitudes of every product term that the
    FP32 accumulation of a split-precision solve adds, i.e. sum_k
    |a_p(i, k)| |b_q(k, r)| over the part products (p, q) that the mode keeps
    (FP32: the float32-rounded operands).  Also returns the number of part
    products per k."""
    from oracle import split
    if mode == "fp32":
        return np.abs(split.round_f32(G)) @ np.abs(split.round_f32(rho_cols)), 1
    parts = {"bf16x3": 2, "bf16x6": 3}[mode]
    a = [np.abs(x) for x in split.split_bf16(G, parts)]
    b = [np.abs(x) for x in split.split_bf16(rho_cols, parts)]
    pairs = [(p, q) for p in range(parts) for q in range(parts) if p + q <= parts - 1]
    return sum(a[p] @ b[q] for p, q in pairs), len(pairs)


def split_elementwise_bound(G, rho_cols, mode, h):
    """Per-entry bound on |u_gpu - u_emulated| for a split-precision solve.

    The GPU and the oracle's emulation multiply the same split parts exactly
    and differ only in how the products are added: the GPU in FP32 (each
    matrix-core accumulation rounds to 24 bits; split-k parts and the leading
    and correction sums are added in FP64), the emulation in FP64.  With
    n = K * (part products per k) FP32 roundings, each at most 2^-24 times a
    partial sum bounded by T (split_term_magnitudes), the error is a sum of n
    such terms; their statistical size sqrt(n) 2^-24 T is taken as the bound
    (the worst case n 2^-24 T is far looser), times h^2 for the scaling."""
    T, npairs = split_term_magnitudes(G, rho_cols, mode)
    K = G.shape[1]
    return (h * h) * np.sqrt(K * npairs) * 2.0 ** -24 * T


def split_tolerances(G, rho_cols, mode):
    """Per-RHS bound on the relative L2 error of a split-precision solve
    against FP64, derived from the arithmetic.

    kappa_r = || |G| |rho_r| || / || G rho_r || measures cancellation in the
    product.  Operand rounding: unit roundoff u_op (2^-24 for FP32; the
    neglected parts of a bfloat16 split are below 2^-16 for 2 parts and 2^-24
    for 3 parts, relative to each operand) gives |error| <= 2 u_op kappa.
    FP32 accumulation adds sqrt(K n) 2^-24 kappa (split_elementwise_bound,
    n part products per k).  Returns an array [R]."""
    A = np.abs(G) @ np.abs(rho_cols)
    U = G @ rho_cols
    kappa = np.linalg.norm(A, axis=0) / np.maximum(np.linalg.norm(U, axis=0), 1e-300)
    u_op = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "bf16x6": 2.0 ** -24}[mode]
    npairs = {"fp32": 1, "bf16x3": 3, "bf16x6": 6}[mode]
    return 2.0 * u_op * kappa + np.sqrt(G.shape[1] * npairs) * 2.0 ** -24 * kappa


def check_split_solve(u_cols, G, rho_cols, h, mode, ref64=None, emu=None, separation=0.5, literal=True):
    """The checks of a split-precision solve u_cols [N, R]:
    (1) element by element within split_elementwise_bound of the oracle's
    exact-product emulation (plus four FP64 roundings of the result);
    (2) per right-hand side within split_tolerances of the FP64 solve;
    (3) for FP32 and BF16x6, mode separation from BF16x3, per right-hand
    side: the distance to the mode's own exact emulation is at most
    ``separation`` times the distance to the exact BF16x3 emulation, and
    (``literal``) the error against FP64 is at most ``separation`` times the
    emulated BF16x3 solve's.  A kernel that dropped the extra part products
    computes BF16x3 and fails (3).  Where the data has little cancellation
    (smooth positive right-hand sides) FP32 accumulation errors are of the
    size of BF16x3's operand error, so there the caller asks only that the
    result be nearer its own emulation (separation = 1, literal = False).
    Returns the per-RHS relative L2 errors against FP64; raises
    AssertionError."""
    from oracle import metrics, split
    if ref64 is None:
        ref64 = apply.plain_apply(G, rho_cols, h)
    if emu is None:
        emu = split.split_apply(G, rho_cols, h, mode)
    bound = split_elementwise_bound(G, rho_cols, mode, h) + 4 * 2.0 ** -53 * np.abs(emu)
    diff = np.abs(u_cols - emu)
    assert np.all(diff <= bound), f"{mode}: max |u - emulation| / bound = {np.max(diff / np.maximum(bound, 1e-300)):.3g}"
    err = metrics.rel_l2_per_rhs(u_cols, ref64)
    tol = split_tolerances(G, rho_cols, mode)
    assert np.all(err <= tol), f"{mode}: max rel L2 / bound vs FP64 = {np.max(err / tol):.3g}"
    if mode in ("fp32", "bf16x6"):
        emu3 = split.split_apply(G, rho_cols, h, "bf16x3")
        near = metrics.rel_l2_per_rhs(u_cols, emu) / np.maximum(metrics.rel_l2_per_rhs(u_cols, emu3), 1e-300)
        assert np.all(near <= separation), f"{mode}: max |u - own emulation| / |u - bf16x3 emulation| = {near.max():.3g}"
        if literal:
            err3 = metrics.rel_l2_per_rhs(emu3, ref64)
            assert np.all(err <= separation * err3), f"{mode}: max err / emulated bf16x3 err = {np.max(err / err3):.3g}"
    return err
