"""Benchmark: solves/s of the quantised (int8 digit-slice matrix-core) form
against the plain FP64 GEMM form of the dense-inverse Poisson solve, on one
MI355X, at 128x128 grid points (126^2 = 15876 unknowns) with 1024 uniform[-1,1]
right-hand sides.

One step = one apply of the precomputed inverse to the 1024-RHS batch: the
int8 form quantises rho to 16-bit fixed point, runs the 6 slice-pair products
of the 24-bit inverse on the int8 matrix cores and recombines them exactly;
the FP64 form is one FP64 matrix-core GEMM.  Inputs are resident in HBM when
the timed region starts; setup (GPU Cholesky inversion, quantisation of G) is
timed separately and never folded into solves/s.

Prints one JSON line.  `value` is the int8 form's solves/s.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0     # MI355X dense int8 matrix peak, TOP/s
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 matrix peak, TFLOP/s
PEAK_HBM_GBS = 8000.0
# the FP64 apply for many right-hand sides: a packing pass over rho, then the
# one-wave-per-SIMD 256 x 128 tile GEMM (timed together)
FP64_APPLY_KERNEL = "apply_f64_w4_kernel (with pack_rhs_kernel)"


def _src_hash(rel):
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(summary, kernel_src, variant=None):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it was
    taken on the current kernel source (and, for the int8 kernel, on the
    variant this run uses); else None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_sha256_16") != _src_hash(kernel_src):
            return None
        if variant is not None:
            by = d.get("hbm_bytes_per_launch_by_variant", {})
            return float(by[str(variant)]) if str(variant) in by else None
        return float(d["hbm_bytes_per_launch"])
    except Exception:
        return None


def _cpu_baseline(wl, bits, rho_bits, nsample, u_gpu):
    """The oracle's applies on a sample of the right-hand sides, on the host's
    cores: the integer apply that the headline value computes (quantise rho,
    exact int64 product with the quantised inverse, scaling) and the plain
    FP64 apply (library matmul), each on every core this process may use and
    on one core.  The integer apply runs as independent column blocks on a
    thread pool (numpy releases the interpreter lock inside the product); the
    FP64 apply's BLAS gets its thread count from threadpoolctl.  The GPU's
    output on the sample is checked bit for bit against the integer apply."""
    import concurrent.futures
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import apply, inverse, quant
    n, h, rho = wl["n"], wl["h"], wl["rho"]
    ncores = len(os.sched_getaffinity(0))
    G = inverse.dst_inverse(n, n)
    S, Sr = bits // 8, rho_bits // 8
    qG, e = quant.quantize_rows(G, S)
    sample = np.ascontiguousarray(rho[:nsample].T)

    def integer_block(cols):
        qR, f = quant.quantize_cols(sample[:, cols], Sr)
        return apply.integer_apply(qG, e, S, qR, f, Sr, h)[0]

    def integer(threads):
        blocks = [b for b in np.array_split(np.arange(nsample), threads) if b.size]
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            with concurrent.futures.ThreadPoolExecutor(len(blocks)) as ex:
                parts = list(ex.map(integer_block, blocks))
            dt = time.perf_counter() - t0
        return np.concatenate(parts, axis=1), dt

    # the FP64 apply is timed on more right-hand sides (it is ~10x faster)
    nf = min(rho.shape[0], 8 * nsample)
    sample64 = np.ascontiguousarray(rho[:nf].T)

    def fp64(threads):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            apply.plain_apply(G, sample64, h)
            return time.perf_counter() - t0

    u_all, t_int_all = integer(ncores)
    _, t_int_1 = integer(1)
    t_f64_all = fp64(ncores)
    t_f64_1 = fp64(1)
    exact = bool(np.array_equal(u_all, u_gpu[:nsample].T))

    def rate(dt, threads, what, cols=nsample):
        return {"value": cols / dt, "unit": "solves/s", "threads": threads, "seconds": dt, "right_hand_sides": cols,
                "what": what}

    int_what = (f"quantise rho to {rho_bits}-bit, exact int64 product with the {bits}-bit per-row inverse, "
                f"scaling (numpy int64 matmul)")
    f64_what = "u = -h^2 G rho in float64 (OpenBLAS matmul)"
    return dict(value=nsample / t_int_all, unit="solves/s", cores=ncores, kind="oracle",
                sample=f"{nsample} of {rho.shape[0]} right-hand sides of the same batch; the oracle's integer apply "
                       f"(the headline arithmetic) on all {ncores} cores; also its integer apply on 1 core and its "
                       f"FP64 apply ({nf} right-hand sides) on {ncores} cores and on 1 core",
                nproc=ncores,
                integer_all_cores=rate(t_int_all, ncores, int_what),
                integer_1_core=rate(t_int_1, 1, int_what),
                fp64_all_cores=rate(t_f64_all, ncores, f64_what, nf),
                fp64_1_core=rate(t_f64_1, 1, f64_what, nf)), exact


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nrhs", type=int, default=1024)
    ap.add_argument("--bits", type=int, default=24)
    ap.add_argument("--rho-bits", type=int, default=16)
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="use the default int8 kernel variant")
    ap.add_argument("--int8-variant", type=int, default=None,
                    help="use this int8 kernel variant instead of autotuning (profiling runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for HBM byte counters)")
    ap.add_argument("--workload", default="quant_128",
                    choices=["quant_128", "plain_32", "vareps_64", "grad_192", "batched", "coupled_32", "gemv_128",
                             "poisson3d_26", "split_128"],
                    help="quant_128 is the headline metric; the others measure the remaining paths")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the dense-inverse apply is measured on a single MI355X "
              "(multi-GPU row-block sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1602_00001_amd import pinv, workloads

    torch.cuda.set_device(0)
    if args.workload != "quant_128":
        print(json.dumps(OTHER[args.workload](args)), flush=True)
        return
    wl = workloads.quant_128(args.nrhs)
    n, h = wl["n"], wl["h"]
    N = (n - 2) * (n - 2)
    R = args.nrhs
    S, Sr = args.bits // 8, args.rho_bits // 8

    t0 = time.perf_counter()
    op = pinv.PoissonInverse.build(n, n, h)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    op.quantize(args.bits)
    torch.cuda.synchronize()
    t_quant = time.perf_counter() - t0
    rho = torch.from_numpy(wl["rho"]).cuda()
    t0 = time.perf_counter()
    variant, variant_ms = _autotune(op, args, args.rho_bits, rho)
    t_tune = time.perf_counter() - t0

    u8 = torch.empty_like(rho)
    u64 = torch.empty_like(rho)
    for _ in range(args.warmup):
        op.apply(rho, "int8", args.rho_bits, out=u8)
        op.apply(rho, "fp64", out=u64)
    torch.cuda.synchronize()
    for k in ("gemm_i8", "quantize_cols", "gemm_f64"):
        pinv.trace_read(k)

    # ---- timed: int8 form (the metric) ----
    pinv.trace_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.apply(rho, "int8", args.rho_bits, out=u8)
    torch.cuda.synchronize()
    t_int8 = time.perf_counter() - t0
    # ---- timed: FP64 GEMM form (the comparison) ----
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.apply(rho, "fp64", out=u64)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    pinv.trace_enable(False)
    gi8_each, gi8_n = pinv.trace_read_each("gemm_i8")
    gi8_ms = sum(gi8_each)
    qc_ms, qc_n = pinv.trace_read("quantize_cols")
    gf_each, gf_n = pinv.trace_read_each("gemm_f64")
    gf_ms = sum(gf_each)

    # accuracy of the quantised form against FP64 on this batch
    diff = torch.linalg.vector_norm(u8 - u64, dim=1) / torch.linalg.vector_norm(u64, dim=1)
    rel_l2_max = float(diff.max())
    rel_l2_med = float(diff.median())

    ms_step = 1e3 * t_int8 / args.steps
    int8_sps = R * args.steps / t_int8
    fp64_sps = R * args.steps / t_fp64

    gi8_avg = gi8_ms / max(gi8_n, 1)
    ops = 2.0 * S * Sr * N * N * R
    ach_i8 = ops / (gi8_avg * 1e-3) / 1e12
    gf_avg = gf_ms / max(gf_n, 1)
    flops = 2.0 * N * N * R
    ach_f64 = flops / (gf_avg * 1e-3) / 1e12

    line = {
        "metric": "solves/sec at 126^2 unknowns: int8-slice MFMA vs FP64 GEMM at <=1e-4 rel L2",
        "value": int8_sps,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {
            "workload": f"quant_128: 128x128 grid, {N} interior unknowns, eps=1, {R} uniform[-1,1] RHS, "
                        f"{args.bits}-bit per-row inverse x {args.rho_bits}-bit rho ({S * Sr} int8 slice pairs)",
            "n_unknowns": N, "nrhs": R, "inverse_bits": args.bits, "rho_bits": args.rho_bits,
        },
        "fp64_gemm": {"value": fp64_sps, "unit": "solves/s", "ms_per_step": 1e3 * t_fp64 / args.steps},
        "int8_over_fp64": int8_sps / fp64_sps,
        "rel_l2_vs_fp64": {"max": rel_l2_max, "median": rel_l2_med, "bound": 1e-4, "ok": rel_l2_max <= 1e-4},
        "roofline": {
            "kernel": f"gemm_i8_kernel<{S},{Sr}> variant {variant}",
            "bound": "mfma", "achieved": ach_i8, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
            "frac": ach_i8 / PEAK_INT8_TOPS,
            "traffic": _traffic("gemm_i8_quant_128.traffic.json", "paper_1602_00001_amd/csrc/gemm_i8.hip", variant),
            "algorithmic_ops_per_launch": ops, "avg_launch_ms": gi8_avg, "launches": gi8_n,
            "median_launch_ms": float(np.median(gi8_each)), "min_launch_ms": min(gi8_each),
            "frac_at_median": ops / (float(np.median(gi8_each)) * 1e-3) / 1e12 / PEAK_INT8_TOPS,
        },
        "roofline_fp64": {
            "kernel": FP64_APPLY_KERNEL,
            "bound": "mfma", "achieved": ach_f64, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": ach_f64 / PEAK_FP64_TFLOPS,
            "traffic": _traffic("gemm_f64_quant_128.traffic.json", "paper_1602_00001_amd/csrc/gemm_f64_apply.hip"),
            "algorithmic_flops_per_launch": flops, "avg_launch_ms": gf_avg, "launches": gf_n,
            "median_launch_ms": float(np.median(gf_each)),
        },
        "quantize_rho_avg_ms": qc_ms / max(qc_n, 1),
        "setup_s": {"build_inverse": t_build, "quantize_inverse": t_quant, "autotune_int8": t_tune},
        "int8_variant": {"chosen": variant, "ms_per_launch": variant_ms},
        "paper_operation_counts": _paper_counts(wl["n"], args.bits, args.rho_bits),
    }
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = nbytes
        del src, dst
    if not args.no_cpu_baseline:
        u_host = u8.cpu().numpy()
        cb, exact = _cpu_baseline(wl, args.bits, args.rho_bits, args.cpu_sample, u_host)
        line["cpu_baseline"] = cb
        line["bit_exact_vs_oracle_on_cpu_sample"] = exact
    else:
        line["cpu_baseline"] = None
    op.close()
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# the other paths (one JSON line each; not the headline metric)

PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0


def _autotune(op, args, rho_bits, rho):
    """Pick the int8 kernel variant for this op on the workload's own right-hand
    sides (setup, outside the timed region)."""
    if args.int8_variant is not None:
        op.set_int8_variant(rho_bits, args.int8_variant)
        return args.int8_variant, None
    if args.no_autotune:
        return 0, None
    return op.autotune_int8(rho_bits, rho=rho, reps=5)


def _paper_counts(n, bits, rho_bits):
    """Operation counts per solve that the paper gives (context, not a target),
    with its N = all n^2 grid nodes and m = 4 decimal digits (the 1e-4 accuracy
    of the metric): Eq. 8 for SOR/Seidel, Eqs. 9-10 for the authors' fast
    product, 2N^2 for a plain matrix-vector product (line 1 of Fig. 4); and the
    integer operations this implementation executes (2 N_interior^2 per digit
    pair)."""
    import math
    N = n * n
    m = 4
    ni = (n - 2) ** 2
    return {"N_nodes": N, "m_digits": m,
            "iterative_eq8": 10.0 * math.log(10.0) / math.pi * m * N * N,
            "fast_product_eq9_eq10": (2.5 + 14.2) * m ** 2.5 * N,
            "dense_matvec_fig4_line1": 2.0 * N * N,
            "this_int8_slices": 2.0 * (bits // 8) * (rho_bits // 8) * ni * ni,
            "note": "elementary operations per right-hand side; the int8 figure counts the 8-bit multiplies and "
                    "adds done on the matrix cores, the paper's figures count scalar operations"}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _base(metric, value, unit, args, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def bench_plain_32(args):
    """One right-hand side on a 32x32 grid: latency of the FP64 GEMV apply."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.plain_32()
    n, h = wl["n"], wl["h"]
    N = (n - 2) ** 2
    op = pinv.PoissonInverse.build(n, n, h)
    rho = torch.from_numpy(wl["rho"]).cuda()
    u = torch.empty_like(rho)
    for _ in range(args.warmup):
        op.apply(rho, "fp64", out=u)
    torch.cuda.synchronize()
    pinv.trace_read("gemv_f64")
    pinv.trace_enable(True)
    dt = _timed(lambda: op.apply(rho, "fp64", out=u), args.steps, 0)
    pinv.trace_enable(False)
    ms, cnt = pinv.trace_read("gemv_f64")
    kms = ms / max(cnt, 1)
    gbs = 8.0 * N * N / (kms * 1e-3) / 1e9
    eager = u.clone()
    # the same time loop captured once in a HIP graph (64 applies) and replayed:
    # no host launch overhead per step
    per_graph = 64
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            op.apply(rho, "fp64", out=u)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            op.apply(rho, "fp64", out=u)
    reps = max(1, args.steps // 4)
    dtg = _timed(graph.replay, reps, 1) / per_graph
    graph_exact = bool(torch.equal(u, eager))
    del graph
    op.close()
    line = _base("solves/sec, 30x30 interior unknowns, one right-hand side, FP64 apply", 1.0 / dt, "solves/s", args,
                 dt * 1e3, "f64", {"workload": "plain_32: 32x32 grid, 900 unknowns, eps=1, 1 blob RHS"})
    line["us_per_solve"] = dt * 1e6
    line["hip_graph"] = {"us_per_solve": dtg * 1e6, "solves_per_s": 1.0 / dtg, "applies_per_graph": per_graph,
                         "bit_identical_to_eager": graph_exact}
    line["roofline"] = {"kernel": "gemv_f64_kernel<1>", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None, "avg_launch_us": kms * 1e3,
                        "note": "the 6.5 MB inverse is cache-resident across steps; launch latency dominates"}
    return line


def bench_coupled_32(args):
    """Time-coupled stepping on 30^2 unknowns: rho_{t+1} = rho_t + tau u_t, one
    right-hand side per step, eager and as a HIP graph of the whole loop."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.coupled_32()
    n, h, tau, steps = wl["n"], wl["h"], wl["tau"], wl["steps"]
    op = pinv.PoissonInverse.build(n, n, h)
    rho0 = torch.from_numpy(wl["rho0"]).cuda()
    r = rho0.clone()
    u = torch.empty_like(r)

    def loop():
        for _ in range(steps):
            op.apply(r, "fp64", out=u)
            r.add_(u, alpha=tau)

    for _ in range(max(args.warmup, 1)):
        r.copy_(rho0)
        loop()
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        r.copy_(rho0)
        loop()
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / (reps * steps)
    eager = r.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        r.copy_(rho0)
        op.apply(r, "fp64", out=u)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        loop()

    def replay():
        r.copy_(rho0)
        graph.replay()

    dt_graph = _timed(replay, reps, 1) / steps
    exact = bool(torch.equal(r, eager))
    del graph
    op.close()
    line = _base("coupled time steps/sec, 30x30 unknowns, one right-hand side per step (FP64 apply + coupling), HIP graph",
                 1.0 / dt_graph, "steps/s", args, dt_graph * 1e3, "f64",
                 {"workload": f"coupled_32: 32x32 grid, 900 unknowns, rho_(t+1) = rho_t + {tau} u_t, {steps} steps per loop"})
    line["us_per_step"] = {"hip_graph": dt_graph * 1e6, "eager": dt_eager * 1e6}
    line["graph_bit_identical_to_eager"] = exact
    return line


def bench_poisson3d_26(args):
    """3-D 7-point operator on a 26^3 grid (24^3 = 13824 unknowns), eps = 1,
    1024 uniform right-hand sides: int8 slices (24-bit x 16-bit) against FP64."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    n, R = 26, 1024
    N = (n - 2) ** 3
    h = 1.0 / (n - 1)
    t0 = time.perf_counter()
    op = pinv.PoissonInverse.build3d(n, n, n, h)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    op.quantize(24)
    rho = torch.from_numpy(workloads.uniform_rhs_n(N, R, workloads.rng(6, 0))).cuda()
    variant, variant_ms = _autotune(op, args, 16, rho)
    u8 = torch.empty_like(rho)
    u64 = torch.empty_like(rho)
    for _ in range(args.warmup):
        op.apply(rho, "int8", 16, out=u8)
        op.apply(rho, "fp64", out=u64)
    torch.cuda.synchronize()
    for k in ("gemm_i8", "gemm_f64"):
        pinv.trace_read(k)
    pinv.trace_enable(True)
    dt8 = _timed(lambda: op.apply(rho, "int8", 16, out=u8), args.steps, 0)
    dt64 = _timed(lambda: op.apply(rho, "fp64", out=u64), args.steps, 0)
    pinv.trace_enable(False)
    gms, gcnt = pinv.trace_read("gemm_i8")
    fms, fcnt = pinv.trace_read("gemm_f64")
    err = torch.linalg.vector_norm(u8 - u64, dim=1) / torch.linalg.vector_norm(u64, dim=1)
    op.close()
    kms8, kms64 = gms / max(gcnt, 1), fms / max(fcnt, 1)
    ach8 = 2.0 * 6 * N * N * R / (kms8 * 1e-3) / 1e12
    ach64 = 2.0 * N * N * R / (kms64 * 1e-3) / 1e12
    line = _base("solves/sec at 24^3 unknowns (3-D 7-point): int8-slice MFMA vs FP64 GEMM", R / dt8, "solves/s", args,
                 dt8 * 1e3, "i8", {"workload": f"poisson3d_26: 26^3 grid, {N} unknowns, eps=1, {R} uniform[-1,1] RHS, "
                                               "24-bit inverse x 16-bit rho"})
    line["fp64_gemm"] = {"value": R / dt64, "unit": "solves/s", "ms_per_step": dt64 * 1e3}
    line["int8_over_fp64"] = dt64 / dt8
    line["rel_l2_vs_fp64"] = {"max": float(err.max()), "median": float(err.median())}
    line["roofline"] = {"kernel": f"gemm_i8_kernel<3,2> variant {variant}", "bound": "mfma", "achieved": ach8,
                        "peak": PEAK_INT8_TOPS, "unit": "TOP/s", "frac": ach8 / PEAK_INT8_TOPS, "traffic": None,
                        "avg_launch_ms": kms8}
    line["roofline_fp64"] = {"kernel": FP64_APPLY_KERNEL, "bound": "mfma", "achieved": ach64,
                             "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach64 / PEAK_FP64_TFLOPS,
                             "avg_launch_ms": kms64}
    line["setup_s"] = {"build_inverse": t_build}
    line["int8_variant"] = {"chosen": variant, "ms_per_launch": variant_ms}
    return line


def bench_gemv_128(args):
    """One right-hand side per call at 126^2 unknowns: the apply is a pass over
    the stored inverse (HBM-bound): FP64 GEMV (2.02 GB), the symmetric-packed
    FP64 copy (1.02 GB), int8 digit planes (24-bit: 0.76 GB) and 16-bit fixed
    point with 64 x 64 tile scales (0.50 GB)."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.quant_128(1)
    n, h = wl["n"], wl["h"]
    N = (n - 2) ** 2
    op = pinv.PoissonInverse.build(n, n, h)
    op.quantize(24)
    op.prepare_split("fp64_sym")
    op.prepare_split("fix16_tile")
    rho = torch.from_numpy(wl["rho"]).cuda()
    u64 = torch.empty_like(rho)
    u8 = torch.empty_like(rho)
    us = torch.empty_like(rho)
    ut = torch.empty_like(rho)
    for _ in range(args.warmup):
        op.apply(rho, "fp64", out=u64)
        op.apply(rho, "int8", 16, out=u8)
        op.apply(rho, "fp64_sym", out=us)
        op.apply(rho, "fix16_tile", out=ut)
    torch.cuda.synchronize()
    for k in ("gemv_f64", "gemv_i8", "quantize_cols", "gemv_sym", "gemv_tile16"):
        pinv.trace_read(k)
    pinv.trace_enable(True)
    dt64 = _timed(lambda: op.apply(rho, "fp64", out=u64), args.steps, 0)
    dt8 = _timed(lambda: op.apply(rho, "int8", 16, out=u8), args.steps, 0)
    dts = _timed(lambda: op.apply(rho, "fp64_sym", out=us), args.steps, 0)
    dtt = _timed(lambda: op.apply(rho, "fix16_tile", out=ut), args.steps, 0)
    pinv.trace_enable(False)
    fms, fcnt = pinv.trace_read("gemv_f64")
    ims, icnt = pinv.trace_read("gemv_i8")
    sms, scnt = pinv.trace_read("gemv_sym")
    tms, tcnt = pinv.trace_read("gemv_tile16")
    err = float(torch.linalg.vector_norm(u8 - u64) / torch.linalg.vector_norm(u64))
    err_sym = float(torch.linalg.vector_norm(us - u64) / torch.linalg.vector_norm(u64))
    err_t = float(torch.linalg.vector_norm(ut - u64) / torch.linalg.vector_norm(u64))
    op.close()
    k64 = fms / max(fcnt, 1)
    k8 = ims / max(icnt, 1)
    gbs64 = (8.0 * N * N + 16.0 * N) / (k64 * 1e-3) / 1e9
    gbs8 = (3.0 * N * N + 10.0 * N) / (k8 * 1e-3) / 1e9
    line = _base("solves/sec at 126^2 unknowns, one RHS per call (FP64 GEMV over the stored inverse)", 1.0 / dt64,
                 "solves/s", args, dt64 * 1e3, "f64",
                 {"workload": f"gemv_128: 128x128 grid, {N} unknowns, eps=1, 1 uniform[-1,1] RHS per call"})
    line["roofline"] = {"kernel": "gemv_f64_kernel<1>", "bound": "hbm", "achieved": gbs64, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": gbs64 / PEAK_HBM_GBS, "traffic": None, "avg_launch_ms": k64}
    nb = (N + 63) // 64
    ks = sms / max(scnt, 1)
    sym_bytes = 8.0 * (nb * (nb + 1) // 2) * 64 * 64 + 2 * 8.0 * nb * nb * 64 + 16.0 * N
    line["fp64_sym"] = {"value": 1.0 / dts, "unit": "solves/s", "ms_per_step": dts * 1e3, "rel_l2_vs_fp64": err_sym,
                        "roofline": {"kernel": "sym_block_kernel<1> + sym_reduce_kernel", "bound": "hbm",
                                     "achieved": sym_bytes / (ks * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                     "frac": sym_bytes / (ks * 1e-3) / 1e9 / PEAK_HBM_GBS, "avg_launch_ms": ks,
                                     "bytes": "packed upper-triangle blocks + block partials written and read"}}
    kt = tms / max(tcnt, 1)
    t16_bytes = 2.0 * N * N + 4.0 * nb * nb + 16.0 * N
    line["fix16_tile"] = {"value": 1.0 / dtt, "unit": "solves/s", "ms_per_step": dtt * 1e3, "rel_l2_vs_fp64": err_t,
                          "roofline": {"kernel": "gemv_tile16_kernel<1>", "bound": "hbm",
                                       "achieved": t16_bytes / (kt * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                                       "unit": "GB/s", "frac": t16_bytes / (kt * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                       "avg_launch_ms": kt,
                                       "bytes": "int16 entries + tile exponents + rho read + u written"}}
    line["int8"] = {"value": 1.0 / dt8, "unit": "solves/s", "ms_per_step": dt8 * 1e3, "rel_l2_vs_fp64": err,
                    "roofline": {"kernel": "gemv_i8_kernel<3,2,1>", "bound": "hbm",
                                 "achieved": gbs8, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs8 / PEAK_HBM_GBS,
                                 "avg_launch_ms": k8}}
    return line


def bench_vareps_64(args):
    """64x64 grid, variable eps, 256 drifting-blob time steps: FP64 against the
    FP32 and BF16 split forms."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.vareps_64()
    n, h = wl["n"], wl["h"]
    N = (n - 2) ** 2
    R = wl["rho"].shape[0]
    op = pinv.PoissonInverse.build(n, n, h, wl["eps"])
    rho = torch.from_numpy(wl["rho"]).cuda()
    ref = op.apply(rho, "fp64")
    # cold-cache timing: 1 GiB written between applies evicts L2 and the
    # 256 MB Infinity Cache; events bracket the apply alone
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")

    def cold_ms(fn, reps):
        times = []
        for _ in range(reps):
            flush.fill_(1.0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return sorted(times)[len(times) // 2]

    modes = {}
    for mode, kern, prods, peak, unit in (("fp64", "gemm_f64", 1, PEAK_FP64_TFLOPS, "TFLOP/s"),
                                          ("fp32", "gemm_split", 1, PEAK_FP32_TFLOPS, "TFLOP/s"),
                                          ("bf16x3", "gemm_split", 3, PEAK_BF16_TFLOPS, "TFLOP/s"),
                                          ("bf16x6", "gemm_split", 6, PEAK_BF16_TFLOPS, "TFLOP/s")):
        if mode != "fp64":
            op.prepare_split(mode)
        u = torch.empty_like(rho)
        for _ in range(args.warmup):
            op.apply(rho, mode, out=u)
        torch.cuda.synchronize()
        pinv.trace_read(kern)
        pinv.trace_enable(True)
        dt = _timed(lambda: op.apply(rho, mode, out=u), args.steps, 0)
        pinv.trace_enable(False)
        ms, cnt = pinv.trace_read(kern)
        kms = ms / max(cnt, 1)
        cms = cold_ms(lambda: op.apply(rho, mode, out=u), max(5, min(args.steps, 20)))
        ach = 2.0 * prods * N * N * R / (kms * 1e-3) / 1e12
        err = torch.linalg.vector_norm(u - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)
        modes[mode] = {"solves_per_s": R / dt, "ms_per_step": dt * 1e3, "kernel_ms": kms,
                       "cold_cache": {"ms_per_step": cms, "solves_per_s": R / (cms * 1e-3)},
                       "rel_l2_vs_fp64_max": float(err.max()), "rel_l2_vs_fp64_median": float(err.median()),
                       "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}}
    op.close()
    best = max(modes, key=lambda m: modes[m]["solves_per_s"])
    line = _base("solves/sec at 62^2 unknowns, variable eps: FP64 vs FP32 / BF16x3 / BF16x6 split precision",
                 modes["bf16x3"]["solves_per_s"], "solves/s", args, modes["bf16x3"]["ms_per_step"], "bf16",
                 {"workload": f"vareps_64: 64x64 grid, {N} unknowns, eps=1+0.5 sin(2 pi x) cos(2 pi y), {R} drifting-blob RHS"})
    line["modes"] = modes
    line["fastest_mode"] = best
    line["roofline"] = dict(modes["bf16x3"]["roofline"], kernel="gemm_bf16_kernel<2>", traffic=None)
    line["note"] = ("the 118 MB FP64 inverse (30 MB per bf16 part) fits the 256 MB Infinity Cache: value and "
                    "ms_per_step are warm-cache rates; cold_cache times one apply after 1 GiB of writes (median)")
    return line


def bench_grad_192(args):
    """192x192 grid: forward (16-bit quantised) + adjoint + eps-gradient of the
    sampled-point loss, 256 right-hand sides per step."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.grad_192()
    n, h = wl["n"], wl["h"]
    N = (n - 2) ** 2
    R = wl["rho"].shape[0]
    t0 = time.perf_counter()
    op = pinv.PoissonInverse.build(n, n, h, wl["eps"])
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    op.quantize(16, keep_fp64=False)
    rho = torch.from_numpy(wl["rho"]).cuda()
    variant, variant_ms = _autotune(op, args, 16, rho)
    idx = torch.from_numpy(wl["sample"]).cuda()
    d = torch.randn(R, idx.numel(), dtype=torch.float64, device="cuda") * 1e-3
    u = torch.empty_like(rho)
    gu = torch.zeros_like(rho)
    lam = torch.empty_like(rho)
    ge = torch.empty((n, n), dtype=torch.float64, device="cuda")

    def step():
        op.apply(rho, "int8", 16, out=u)
        gu[:, idx] = 2.0 * (u[:, idx] - d)
        op.apply_adjoint(gu, "int8", 16, out=lam)
        op.grad_eps(u, lam, out=ge)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in ("gemm_i8", "grad_eps", "quantize_cols"):
        pinv.trace_read(k)
    pinv.trace_enable(True)
    dt = _timed(step, args.steps, 0)
    pinv.trace_enable(False)
    gms, gcnt = pinv.trace_read("gemm_i8")
    ems, ecnt = pinv.trace_read("grad_eps")
    qms, qcnt = pinv.trace_read("quantize_cols")
    kms = gms / max(gcnt, 1)
    ops = 2.0 * 4 * N * N * R
    ach = ops / (kms * 1e-3) / 1e12
    op.close()
    line = _base("right-hand sides/sec through forward + adjoint + eps-gradient at 190^2 unknowns (16-bit)",
                 R / dt, "rhs/s", args, dt * 1e3, "i8",
                 {"workload": f"grad_192: 192x192 grid, {N} unknowns, eps=1+0.5 sin cos, {R} blob RHS, 512 sampled points, 16-bit inverse x 16-bit rho/g"})
    line["roofline"] = {"kernel": f"gemm_i8_kernel<2,2> variant {variant}", "bound": "mfma", "achieved": ach,
                        "peak": PEAK_INT8_TOPS,
                        "unit": "TOP/s", "frac": ach / PEAK_INT8_TOPS, "traffic": None, "avg_launch_ms": kms}
    line["grad_eps_avg_ms"] = ems / max(ecnt, 1)
    line["quantize_avg_ms"] = qms / max(qcnt, 1)
    line["setup_s"] = {"build_inverse": t_build}
    line["int8_variant"] = {"chosen": variant, "ms_per_launch": variant_ms}
    return line


def bench_batched(args):
    """4096 requests over 20 operators (grids 32^2..160^2, 4 log-normal eps fields
    per size), 1-64 blob right-hand sides each, 16-bit quantised, one batched call."""
    import numpy as np
    import torch
    from paper_1602_00001_amd import pinv, workloads
    opdefs, reqs = workloads.batched_requests()
    t0 = time.perf_counter()
    ops = []
    for od in opdefs:
        n = od["n"]
        op = pinv.PoissonInverse.build(n, n, 1.0 / (n - 1), od["eps"])
        op.quantize(16, keep_fp64=False)
        ops.append(op)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    batch = []
    total_rhs = 0
    ops_count = 0.0
    for r in reqs:
        op = ops[r["op"]]
        n = opdefs[r["op"]]["n"]
        par = workloads.blob_params_batch(np.random.default_rng(r["seed"]), r["nrhs"])
        rho = workloads.blob_rhs_device(n, par)
        batch.append((op, rho, torch.empty_like(rho)))
        total_rhs += r["nrhs"]
        ops_count += 2.0 * 4 * op.n * op.n * r["nrhs"]
    # the first call plans the request list (device tables, scratch, and each
    # grouped launch's kernel variant timed on the launch itself)
    t0 = time.perf_counter()
    pinv.apply_batched(batch, "int8", 16)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    for _ in range(args.warmup):
        pinv.apply_batched(batch, "int8", 16)
    torch.cuda.synchronize()
    for k in ("gemm_i8", "quantize_cols"):
        pinv.trace_read(k)
    pinv.trace_enable(True)
    dt = _timed(lambda: pinv.apply_batched(batch, "int8", 16), args.steps, 0)
    pinv.trace_enable(False)
    gms, gcnt = pinv.trace_read("gemm_i8")
    qms, qcnt = pinv.trace_read("quantize_cols")
    steps_traced = args.steps
    gemm_ms_per_step = gms / steps_traced
    ach = ops_count / (gemm_ms_per_step * 1e-3) / 1e12
    for op in ops:
        op.close()
    line = _base("solves/sec over 4096 uneven requests (grids 32^2..160^2, 1-64 RHS each), 16-bit quantised, grouped by operator",
                 total_rhs / dt, "solves/s", args, dt * 1e3, "i8",
                 {"workload": f"batched: {len(reqs)} requests, {len(opdefs)} operators, {total_rhs} right-hand sides"})
    line["roofline"] = {"kernel": "grouped int8 slice GEMM <2,2> (all groups, one launch)", "bound": "mfma", "achieved": ach,
                        "peak": PEAK_INT8_TOPS, "unit": "TOP/s", "frac": ach / PEAK_INT8_TOPS, "traffic": None,
                        "gemm_ms_per_step": gemm_ms_per_step, "gemm_launches_per_step": gcnt / steps_traced}
    line["quantize_ms_per_step"] = qms / steps_traced
    line["setup_s"] = {"build_and_quantize_20_operators": t_setup, "plan_and_tune_first_call": t_plan}
    return line


def bench_split_128(args):
    """The split-precision forms (FP32, BF16x3, BF16x6) at the metric's size,
    126^2 unknowns x 1024 uniform right-hand sides, against FP64: the split
    kernels on a problem large enough to fill the chip without splitting k
    (the 62^2 x 256 workload is a few tens of microseconds of work)."""
    import torch
    from paper_1602_00001_amd import pinv, workloads
    wl = workloads.quant_128(1024)
    n, h = wl["n"], wl["h"]
    N = (n - 2) ** 2
    R = wl["rho"].shape[0]
    op = pinv.PoissonInverse.build(n, n, h)
    rho = torch.from_numpy(wl["rho"]).cuda()
    ref = op.apply(rho, "fp64")
    modes = {}
    for mode, kern, prods, peak, unit in (("fp64", "gemm_f64", 1, PEAK_FP64_TFLOPS, "TFLOP/s"),
                                          ("fp32", "gemm_split", 1, PEAK_FP32_TFLOPS, "TFLOP/s"),
                                          ("bf16x3", "gemm_split", 3, PEAK_BF16_TFLOPS, "TFLOP/s"),
                                          ("bf16x6", "gemm_split", 6, PEAK_BF16_TFLOPS, "TFLOP/s")):
        if mode != "fp64":
            op.prepare_split(mode)
        u = torch.empty_like(rho)
        for _ in range(args.warmup):
            op.apply(rho, mode, out=u)
        torch.cuda.synchronize()
        pinv.trace_read(kern)
        pinv.trace_enable(True)
        dt = _timed(lambda: op.apply(rho, mode, out=u), args.steps, 0)
        pinv.trace_enable(False)
        ms, cnt = pinv.trace_read(kern)
        kms = ms / max(cnt, 1)
        ach = 2.0 * prods * N * N * R / (kms * 1e-3) / 1e12
        err = torch.linalg.vector_norm(u - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)
        modes[mode] = {"solves_per_s": R / dt, "ms_per_step": dt * 1e3, "kernel_ms": kms,
                       "rel_l2_vs_fp64_max": float(err.max()), "rel_l2_vs_fp64_median": float(err.median()),
                       "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}}
    op.close()
    line = _base("solves/sec at 126^2 unknowns, 1024 RHS: FP64 vs FP32 / BF16x3 / BF16x6 split precision",
                 modes["bf16x3"]["solves_per_s"], "solves/s", args, modes["bf16x3"]["ms_per_step"], "bf16",
                 {"workload": f"split_128: 128x128 grid, {N} unknowns, eps=1, {R} uniform[-1,1] RHS"})
    line["modes"] = modes
    line["roofline"] = dict(modes["bf16x3"]["roofline"], kernel="gemm_i8_kernel<2,2,...,1> (bf16 parts)", traffic=None)
    return line


OTHER = {"plain_32": bench_plain_32, "vareps_64": bench_vareps_64, "grad_192": bench_grad_192,
         "batched": bench_batched, "coupled_32": bench_coupled_32, "poisson3d_26": bench_poisson3d_26,
         "gemv_128": bench_gemv_128, "split_128": bench_split_128}


if __name__ == "__main__":
    main()
