"""Pins of the split-precision emulation: bfloat16 rounding against torch's own
float32 -> bfloat16 conversion (an independent library routine), exactness of
the residuals, and the error envelope of each mode."""

import numpy as np
import pytest
import torch

from oracle import apply, grid, inverse, metrics, split


def test_round_bf16_matches_torch_on_float32_values():
    g = np.random.default_rng(0)
    x = (g.standard_normal(20000) * np.exp(g.uniform(-20, 20, 20000))).astype(np.float32)
    # include exact ties: 1 + (2k+1) 2^-8
    ties = (1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8).astype(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, 1.0, -3.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    ours = split.round_bf16(x.astype(np.float64))
    assert np.array_equal(ours, ref)


def test_split_residuals_exact_and_decreasing():
    g = np.random.default_rng(1)
    x = g.standard_normal(5000)
    parts = split.split_bf16(x, 3)
    rest = x - parts[0] - parts[1] - parts[2]
    assert np.all(np.abs(parts[1]) <= np.abs(x) * 2.0 ** -8)
    assert np.all(np.abs(rest) <= np.abs(x) * 2.0 ** -24)
    # each part is a bfloat16 value
    for p in parts:
        assert np.array_equal(split.round_bf16(p), p)


@pytest.mark.parametrize("mode,tol", [("fp32", 5e-7), ("bf16x3", 3e-5), ("bf16x6", 1e-6)])
def test_split_modes_error_envelope(mode, tol):
    n = 30
    K, _ = grid.conservative_operator(n, n)
    G = inverse.lu_inverse(K)
    h = 1.0 / (n - 1)
    rho = np.random.default_rng(2).uniform(-1, 1, (G.shape[0], 6))
    ref = apply.plain_apply(G, rho, h)
    u = split.split_apply(G, rho, h, mode)
    err = np.max(metrics.rel_l2_per_rhs(u, ref))
    assert err < tol
