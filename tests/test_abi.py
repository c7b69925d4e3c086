"""The C-ABI boundary without a GPU: the shared library loads, exports every
function include/ppe.h declares, the Python binding declares exactly those
functions, and every field of the public structs sits at the same offset in
the binding as in a C compile of the header (gcc, offsetof)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2604_01800_amd import ppe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppe.h")
STRUCTS = ["ppe_grid_desc", "ppe_solve_opts", "ppe_solve_stats", "ppe_net_config", "ppe_train_opts",
           "ppe_tune_result", "ppe_net_tune_result"]


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ppe_[a-z0-9_]+)\s*\(", text)))


def library():
    path = ppe.LIB_PATH
    if not os.path.exists(path):
        from paper_2604_01800_amd import build
        build.build()
    return ctypes.CDLL(path)


def test_library_exports_every_declared_function():
    L = library()
    names = declared_functions()
    assert len(names) >= 20, names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_declares_exactly_the_header():
    assert set(ppe.SIGNATURES) == set(declared_functions())


def test_enum_values_match_header():
    text = open(HEADER).read()
    for name in ["PPE_OK", "PPE_NOT_CONVERGED", "PPE_ERR_INVALID_ARG", "PPE_ERR_SHAPE", "PPE_ERR_UNSUPPORTED",
                 "PPE_ERR_HIP", "PPE_ERR_NONFINITE", "PPE_PC_NONE", "PPE_PC_JACOBI", "PPE_TOL_RELATIVE",
                 "PPE_TOL_ABSOLUTE", "PPE_PCG_AUTO", "PPE_PCG_SINGLE_REDUCTION", "PPE_PCG_TWO_PHASE", "PPE_PCG_TWO_STEP",
                 "PPE_DIR_NET",
                 "PPE_DIR_ZERO", "PPE_DIR_JACOBI", "PPE_DIR_NAN", "PPE_DIR_ONES"]:
        m = re.search(r"\b" + name + r"\s*=\s*(-?\d+)", text)
        assert m, name
        assert int(m.group(1)) == getattr(ppe, name), name


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_struct_layout_matches_c(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ppe.h"', "int main(void) {"]
    expect = []
    for s in STRUCTS:
        cls = getattr(ppe, s)
        lines.append(f'  printf("%zu\\n", sizeof({s}));')
        expect.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({s}, {fname}));')
            expect.append(getattr(cls, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = ["-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include"]
    subprocess.run(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", *inc, "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_noalloc_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define\s+PPE_NOALLOC_SCRATCH_BYTES\s+\(([^)]*)\)", text)
    assert m, "PPE_NOALLOC_SCRATCH_BYTES not defined"
    assert eval(m.group(1), {}, {}) == ppe.PPE_NOALLOC_SCRATCH_BYTES
