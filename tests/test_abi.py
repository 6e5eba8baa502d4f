"""The C-ABI library loads and exports every function include/dtsdf.h declares (no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dtsdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dtsdf_create", "dtsdf_destroy", "dtsdf_integrate", "dtsdf_render", "icp_step",
              "dtsdf_export", "dtsdf_import", "dtsdf_status_string"]:
        assert n in names, names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2301_12796_amd", "libdtsdf.so"))
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_status_strings_without_device():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2301_12796_amd", "libdtsdf.so"))
    lib.dtsdf_status_string.restype = ctypes.c_char_p
    assert lib.dtsdf_status_string(0) == b"ok"
    assert b"invalid" in lib.dtsdf_status_string(1)


def test_binding_declares_the_same_symbols():
    from paper_2301_12796_amd import dtsdf
    assert sorted(dtsdf.EXPORTED) == declared_functions()
