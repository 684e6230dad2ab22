"""The boundary is a plain C interface: include/pinv.h compiles as strict C99
and as C++, a C program that references every declared entry point links
against the built library, and runs (version and status strings only; no
device call)."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1602_00001_amd", "_lib")


def _declared():
    src = open(os.path.join(ROOT, "include", "pinv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pinv_[a-z_0-9]+)\s*\(", src)))


def _program():
    refs = "\n".join(f"  (entry)&{n}," for n in _declared())
    return f"""#include <stdio.h>
#include "pinv.h"

typedef void (*entry)(void);

static const entry entry_points[] = {{
{refs}
}};

int main(void) {{
  pinv_info info;
  pinv_grid grid = {{16, 16, 1.0 / 15.0}};
  (void)info;
  (void)grid;
  printf("%s %s %d\\n", pinv_version(), pinv_status_string(PINV_E_UNSUPPORTED),
         (int)(sizeof(entry_points) / sizeof(entry_points[0])));
  return entry_points[0] == 0;
}}
"""


@pytest.mark.skipif(not os.path.exists(os.path.join(LIBDIR, "libpinv.so")), reason="library not built")
def test_c_program_links_and_runs(tmp_path):
    c = tmp_path / "use_pinv.c"
    c.write_text(_program())
    exe = tmp_path / "use_pinv"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", f"-I{inc}", str(c),
                    f"-L{LIBDIR}", "-lpinv", f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout.split()
    assert out[0] == "0.1.0" or re.match(r"\d+\.\d+\.\d+$", out[0])
    assert int(out[-1]) == len(_declared())


def test_header_compiles_as_cxx(tmp_path):
    cc = tmp_path / "h.cc"
    cc.write_text('#include "pinv.h"\nint main() { return PINV_OK; }\n')
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", f"-I{os.path.join(ROOT, 'include')}", "-fsyntax-only",
                    str(cc)], check=True)
