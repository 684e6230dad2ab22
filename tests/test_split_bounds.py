"""The split-precision parity checks (tests/gpu_util.check_split_solve) on the
CPU, at the sizes the GPU tests use (66^2 with a random eps field, the 62^2
variable-eps workload): solves that add the same split parts in genuine FP32
(numpy float32 products over k chunks of 512, the chunks added in float64, a
different summation order from the GPU's) pass every check, and a BF16x3
solve (exact, or FP32-accumulated like a kernel that dropped the extra part
products) handed to the BF16x6 and FP32 checks is rejected by the mode
separation check."""

import numpy as np
import pytest

from oracle import split
from paper_1602_00001_amd import workloads
from tests.gpu_util import check_split_solve, oracle_inverse


def _cases():
    """(name, G, rho columns, h, check options): the GPU tests' inputs."""
    g = np.random.default_rng(5)
    G, _, _ = oracle_inverse(66, 66, workloads.random_eps(66, 66, g))
    rho = g.uniform(-1, 1, (40, G.shape[0]))
    yield "66x66", G, rho.T, 1.0 / 65, {}
    wl = workloads.vareps_64()
    G, _, _ = oracle_inverse(wl["n"], wl["n"], wl["eps"])
    yield "vareps_64", G, wl["rho"].T, wl["h"], dict(separation=1.0, literal=False)
    rho = np.random.default_rng(6).uniform(-1, 1, (256, G.shape[0]))
    yield "vareps_64 uniform rho", G, rho.T, wl["h"], {}


@pytest.fixture(scope="module")
def cases():
    return list(_cases())


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def fp32_accumulated(G, rho, h, mode, chunk=512):
    """The mode's part products added in float32 over k chunks of ``chunk``
    (leading and correction sums separately), the chunks' sums added in
    float64, as the matrix-core kernels do with their k splits."""
    if mode == "fp32":
        A, B = [[_f32(split.round_f32(G))], [_f32(split.round_f32(rho))]]
        pairs = [(0, 0)]
    else:
        parts = {"bf16x3": 2, "bf16x6": 3}[mode]
        A = [_f32(x) for x in split.split_bf16(G, parts)]
        B = [_f32(x) for x in split.split_bf16(rho, parts)]
        pairs = [(p, q) for p in range(parts) for q in range(parts) if p + q <= parts - 1]
    acc = np.zeros((G.shape[0], rho.shape[1]))
    for k0 in range(0, G.shape[1], chunk):
        ks = slice(k0, k0 + chunk)
        lead = A[0][:, ks] @ B[0][ks]
        corr = np.zeros_like(lead)
        for p, q in pairs[1:]:
            corr += A[p][:, ks] @ B[q][ks]
        acc += lead.astype(np.float64) + corr.astype(np.float64)
    return -(h * h) * acc


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "bf16x6"])
def test_fp32_accumulated_solves_pass(cases, mode):
    for name, G, rho, h, opt in cases:
        err = check_split_solve(fp32_accumulated(G, rho, h, mode), G, rho, h, mode, **opt)
        print(f"[{name}] {mode}: max rel L2 vs FP64 {err.max():.3e}")


@pytest.mark.parametrize("mode", ["fp32", "bf16x6"])
def test_bf16x3_result_is_rejected_as_a_more_accurate_mode(cases, mode):
    for name, G, rho, h, opt in cases:
        for wrong in (split.split_apply(G, rho, h, "bf16x3"), fp32_accumulated(G, rho, h, "bf16x3")):
            with pytest.raises(AssertionError, match="bf16x3"):
                check_split_solve(wrong, G, rho, h, mode, **opt)
