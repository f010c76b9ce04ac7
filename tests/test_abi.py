"""The C-ABI library loads and exports every entry point that include/comm.h
declares (CPU only: no compute calls are made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "comm.h")
LIB = os.path.join(ROOT, "paper_2602_14683_amd", "libcomm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(comm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ["comm_cp_update", "comm_tucker_update", "comm_jcomm_outer", "comm_beta_objective",
                 "comm_cp_jcomm_outer_coo", "comm_create", "comm_destroy", "comm_last_error"]:
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcomm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcomm.so not built")
def test_binding_lists_every_declared_symbol():
    import paper_2602_14683_amd as pkg
    assert sorted(pkg.EXPORTED) == declared_functions()
    assert pkg.load_library() is not None
