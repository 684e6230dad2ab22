"""The C-ABI host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only; the device code is built as usual): _lib/libpinv_san.so is
built from the same sources when missing or older than them, and the
library's host-side checks (tests/test_abi.py) run in a child process that
loads it with the sanitizer runtime preloaded; any sanitizer report aborts the
child.  Runs without a GPU."""

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sources():
    pkg = os.path.join(ROOT, "paper_1602_00001_amd")
    return (glob.glob(os.path.join(pkg, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*.h")) +
            [os.path.join(pkg, "build.py")])


def _fresh_sanitized_library():
    from paper_1602_00001_amd import build as b
    newest = max(os.path.getmtime(f) for f in _sources())
    if not os.path.exists(b.LIB_SAN) or os.path.getmtime(b.LIB_SAN) < newest:
        b.build(sanitize=True)
    return b


def test_library_is_instrumented():
    b = _fresh_sanitized_library()
    syms = subprocess.run(["nm", "-D", "--undefined-only", b.LIB_SAN], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms


def test_host_checks_under_sanitizers():
    b = _fresh_sanitized_library()
    env = b.sanitizer_env()
    probe = subprocess.run([sys.executable, "-c", "from paper_1602_00001_amd import pinv; print(pinv.LIB_PATH)"],
                           env=env, capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert probe.returncode == 0, probe.stderr[-3000:]
    assert probe.stdout.strip() == b.LIB_SAN
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_abi.py")], env=env, capture_output=True, text=True, cwd=ROOT,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "failed" not in r.stdout
