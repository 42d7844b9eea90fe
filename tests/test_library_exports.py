"""The C-ABI library loads without a GPU and exports every call that
include/asm.h declares (no compute calls are made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asm.h")
LIB = os.path.join(ROOT, "paper_1401_7227_amd", "libasm_mi355x.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_1401_7227_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for call in ["asm_create_system", "asm_setup_precond", "asm_solve", "asm_solve_batch",
                 "asm_precond_apply", "asm_spmv", "asm_last_error"]:
        assert call in names


def test_every_declared_call_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_dynamic_symbol_table_matches_binding():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line and line.split()[-1].startswith("asm_")}
    import paper_1401_7227_amd._binding as B
    assert set(B.EXPORTED) <= exported
    assert set(declared_functions()) <= exported


def test_last_error_is_callable_without_gpu(lib):
    lib.asm_last_error.restype = ctypes.c_char_p
    assert lib.asm_last_error() is not None
