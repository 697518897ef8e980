"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ovfem.h")
LIB = os.path.join(ROOT, "paper_2404_13683_amd", "libovfem.so")
PKG = os.path.join(ROOT, "paper_2404_13683_amd")


def _declared():
    text = open(HEADER).read()
    decl = r"^\s*(?:ovfem_status|int32_t|const char\*)\s+(ovfem_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, text, re.M)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libovfem.so not built")


@needs_lib
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


@needs_lib
def test_binding_signatures_cover_the_header():
    from paper_2404_13683_amd import ovfem
    assert sorted(ovfem.SIGNATURES) == _declared()


@needs_lib
def test_invalid_arguments_fail_before_touching_the_device():
    from paper_2404_13683_amd import ovfem
    lib = ovfem.lib()
    h = ctypes.c_void_p()
    assert lib.ovfem_create(None, 4, 4, 4, 1.0, 1, 0, None) == -1
    assert lib.ovfem_create(ctypes.byref(h), 0, 4, 4, 1.0, 1, 0, None) == -1
    assert b"positive" in lib.ovfem_last_error()
    assert lib.ovfem_create(ctypes.byref(h), 4, 4, 4, -1.0, 1, 0, None) == -1
    assert lib.ovfem_create(ctypes.byref(h), 4, 4, 4, 1.0, 1, 7, None) == -1
    assert lib.ovfem_create(ctypes.byref(h), 4, 4, 4, 1.0, 0, 0, None) == -1
    assert lib.ovfem_create(ctypes.byref(h), 4, 4, 4, 1.0, 4097, 0, None) == -1
    assert b"n_shots" in lib.ovfem_last_error()
    # grids beyond the index ranges of the kernels
    assert lib.ovfem_create(ctypes.byref(h), 2048, 2048, 1024, 1.0, 1, 0, None) == -1
    assert b"2^31" in lib.ovfem_last_error()
    assert lib.ovfem_create(ctypes.byref(h), 14000, 14000, 4, 1.0, 1, 0, None) == -1
    assert b"z plane" in lib.ovfem_last_error()
    assert lib.ovfem_step(None, 1) == -1
    assert lib.ovfem_set_tuning(None, 16, 0, 64) == -1
    assert lib.ovfem_autotune(None, 10, None) == -1
    assert lib.ovfem_destroy(None) == 0
    b = ctypes.c_void_p()
    assert lib.ovfem_batch_create(None, None, 1) == -1
    assert lib.ovfem_batch_create(ctypes.byref(b), None, 0) == -1
    members = (ctypes.c_void_p * 1)(None)
    assert lib.ovfem_batch_create(ctypes.byref(b), members, 1) == -1
    assert b"NULL member" in lib.ovfem_last_error()
    assert lib.ovfem_batch_step(None, 1) == -1
    assert lib.ovfem_batch_step_noalloc(None, 1) == -1
    assert b"batch is NULL" in lib.ovfem_last_error()
    assert lib.ovfem_batch_set_tuning(None, 0) == -1
    assert lib.ovfem_batch_set_graph(None, 6) == -1
    assert lib.ovfem_set_tile_rows(None, 16) == -1
    r = ctypes.c_int32()
    assert lib.ovfem_get_tile_rows(None, ctypes.byref(r)) == -1
    assert lib.ovfem_batch_destroy(None) == 0
    assert lib.ovfem_version() >= 200


def test_product_path_does_not_use_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), f
                assert not re.search(r"import_module\(\s*['\"]oracle|#include\s+[<\"][^>\"]*oracle", text), f


@needs_lib
def test_header_is_plain_c_and_links():
    """The header compiles as C99 (no C++ in the ABI), a C program links against the
    library, and its host-side validation answers before any device work."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    work = os.path.join(PKG, "_build", "abi_c_test")  # the package's (ignored) build folder
    os.makedirs(work, exist_ok=True)
    src = os.path.join(work, "abi.c")
    open(src, "w").write(r'''
#include <stdio.h>
#include "ovfem.h"
int main(void) {
  ovfem_solver* s = 0;
  int32_t finite = 0;
  int ok = ovfem_version() >= 200;
  ok &= ovfem_create(0, 4, 4, 4, 1.0, 1, OVFEM_INT8, 0) == OVFEM_EINVAL;
  ok &= ovfem_create(&s, 4, 4, 4, 1.0, 0, OVFEM_FP64, 0) == OVFEM_EINVAL && s == 0;
  ok &= ovfem_step(0, 1) == OVFEM_EINVAL;
  ok &= ovfem_check_finite(0, &finite) == OVFEM_EINVAL;
  printf("%s|", ovfem_last_error());
  ok &= ovfem_destroy(0) == OVFEM_OK;
  printf("%d\n", ok);
  return ok ? 0 : 1;
}
''')
    exe = os.path.join(work, "abi")
    libdir = os.path.dirname(LIB)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), src,
                        "-L", libdir, "-lovfem", "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib",
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "NULL" in run.stdout
