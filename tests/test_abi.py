"""The C-ABI library loads and exports every entry point include/wsest.h
declares; ctypes mirrors of its structs have the C sizes.  No compute calls."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wsest.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wse_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def wlib():
    from paper_2204_14242_amd import wsest
    if not os.path.exists(wsest.LIB_PATH):
        from paper_2204_14242_amd import build
        build.build()
    return wsest


def test_header_declares_the_calls():
    names = declared()
    for n in ("wse_ctx_create", "wse_ctx_destroy", "wse_status_str", "wse_last_error",
              "wse_kernel_register", "wse_hw_register", "wse_space_size", "wse_estimate",
              "wse_rhat", "wse_last_timings"):
        assert n in names


def test_library_exports_every_declared_symbol(wlib):
    L = wlib.lib()
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", wlib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (wse_[a-z_]+)$", out, flags=re.M))
    assert set(declared()) <= exported
    assert set(wlib.exported_symbols()) == set(declared())


def test_status_strings(wlib):
    L = wlib.lib()
    assert L.wse_status_str(0) == b"ok"
    assert L.wse_status_str(-1) == b"invalid argument"
    assert L.wse_status_str(-6) == b"not ready"


def test_struct_sizes_match_the_header(tmp_path):
    from paper_2204_14242_amd import wsest
    src = r'''
#include <stdio.h>
#include "wsest.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(wse_field), sizeof(wse_expr), sizeof(wse_access),
         sizeof(wse_kernel_desc), sizeof(wse_hw), sizeof(wse_space), sizeof(wse_result));
  return 0;
}'''
    c_path = str(tmp_path / "abi_sizes.c")
    exe = str(tmp_path / "abi_sizes")
    open(c_path, "w").write(src)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c_path, "-o", exe], check=True)
    sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes == [C.sizeof(wsest.wse_field), C.sizeof(wsest.wse_expr), C.sizeof(wsest.wse_access),
                     C.sizeof(wsest.wse_kernel_desc), C.sizeof(wsest.wse_hw),
                     C.sizeof(wsest.wse_space), wsest.RESULT_DTYPE.itemsize]


def test_binding_has_no_cpu_fallback():
    # the binding loads the HIP library or raises; it never imports the oracle
    src = open(os.path.join(ROOT, "paper_2204_14242_amd", "wsest.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
