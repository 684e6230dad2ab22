"""Build step of the HIP library: compiles csrc/*.hip for gfx950 and links
_lib/libpinv.so.  Called by ``__graft_entry__.build()`` (and usable as
``python -m paper_1602_00001_amd.build``).

``build(sanitize=True)`` (``python -m paper_1602_00001_amd.build --sanitize``)
makes _lib/libpinv_san.so instead: the same sources with the host code built
under AddressSanitizer and UndefinedBehaviorSanitizer (the device code is
built as usual; sanitizers apply to host code only).  Load it with
PINV_LIBRARY pointing at it and the sanitizer runtime preloaded
(``sanitizer_env()``)."""

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(LIBDIR, "libpinv.so")
LIB_SAN = os.path.join(LIBDIR, "libpinv_san.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-ffp-contract=off",                      # the int8 epilogue's two roundings must stay separate
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-Wno-pass-failed",                       # inner loops whose bounds become constant only once the enclosing loop is unrolled
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# host-only sanitizers: each -fsanitize= goes to the host compilation only
SAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g",
]


def _compile(src, sanitize=False):
    bdir = os.path.join(BUILD, "san") if sanitize else BUILD
    obj = os.path.join(bdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj, errs


def build(verbose=False, sanitize=False):
    out = LIB_SAN if sanitize else LIB
    os.makedirs(os.path.join(BUILD, "san") if sanitize else BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda f: _compile(f, sanitize), srcs))
    for obj, errs in results:
        if verbose and errs.strip():
            print(errs, file=sys.stderr)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    shutil.move(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def sanitizer_runtime():
    """Path of the AddressSanitizer runtime of the compiler that built
    libpinv_san.so (it carries the UndefinedBehaviorSanitizer handlers too)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def sanitizer_env(base=None):
    """Environment for a child process that loads libpinv_san.so."""
    env = dict(os.environ if base is None else base)
    env["PINV_LIBRARY"] = LIB_SAN
    env["LD_PRELOAD"] = sanitizer_runtime()
    # Python's allocator keeps memory until exit; leaks are not this check's
    # subject
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
