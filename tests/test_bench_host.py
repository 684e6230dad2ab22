"""Host-side pieces of the benchmark (no GPU): the paper's operation counts it
quotes, and the rule that an HBM-traffic figure is reported only for the
kernel source and variant it was measured on."""

import importlib.util
import json
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_paper_operation_counts(bench):
    c = bench._paper_counts(128, 24, 16)
    N = 128 * 128
    assert c["N_nodes"] == N and c["m_digits"] == 4
    # Eq. 8: (10 ln 10 / pi) m N^2; Eqs. 9-10: (2.5 + 14.2) m^2.5 N; a plain product 2 N^2
    assert math.isclose(c["iterative_eq8"], 10 * math.log(10) / math.pi * 4 * N * N, rel_tol=1e-12)
    assert math.isclose(c["fast_product_eq9_eq10"], 16.7 * 32.0 * N, rel_tol=1e-12)
    assert c["dense_matvec_fig4_line1"] == 2 * N * N
    assert c["this_int8_slices"] == 2 * 3 * 2 * 126 ** 4


def test_traffic_figure_tied_to_source_and_variant(bench, tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    d = {"kernel_source_sha256_16": bench._src_hash(str(src)), "hbm_bytes_per_launch": 123.0,
         "hbm_bytes_per_launch_by_variant": {"4": 7.0}}
    (prof / "k.traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._traffic("k.traffic.json", str(src)) == 123.0
    assert bench._traffic("k.traffic.json", str(src), variant=4) == 7.0
    assert bench._traffic("k.traffic.json", str(src), variant=8) is None
    src.write_text("// a changed kernel\n")
    assert bench._traffic("k.traffic.json", str(src)) is None
    assert bench._traffic("missing.json", str(src)) is None


def test_more_than_one_gpu_is_refused():
    """bench.py --gpus N with N > 1 exits non-zero with a message saying the
    build runs on one GPU (no GPU touched: the check precedes any device call)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
