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


def test_binding_structs_follow_the_header():
    import paper_2602_14683_amd as pkg
    text = open(HEADER).read()
    assert int(re.search(r"#define COMM_MAX_NDIM (\d+)", text).group(1)) == pkg.MAX_NDIM
    m = re.search(r"#define COMM_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert int(m.group(1)) << int(m.group(2)) == pkg.NOALLOC_SCRATCH_BYTES
    # int + pad + int64[5] + pointer
    assert ctypes.sizeof(pkg.Dense) == 8 + 8 * pkg.MAX_NDIM + 8
    assert ctypes.sizeof(pkg.Model) == 8 + 8 * pkg.MAX_NDIM + 8 * pkg.MAX_NDIM + 8
    # beta, eps, eps_x; inner_sweeps, precision, cache_pq, check_inputs
    assert ctypes.sizeof(pkg.Opts) == 3 * 8 + 4 * 4
    assert [f[0] for f in pkg.Opts._fields_] == re.findall(
        r"^\s+(?:double|int) (\w+);", re.search(r"typedef struct \{\n  double beta;.*?\} comm_opts;", text,
                                                  re.S).group(0), re.M)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcomm.so not built")
def test_workspace_query_by_order():
    """comm_workspace_bytes is host arithmetic only: orders 3 to 5 of dense CP
    and orders 3 to 5 of dense Tucker are accepted, and an order-N tensor whose
    first N - 2 extents multiply past 2^24 is refused (0)."""
    import paper_2602_14683_amd as pkg
    lib = pkg.load_library()

    def ws(dims, rank=0, core=None, beta=1.0, op=1):
        d = pkg.Dense()
        d.ndim = len(dims)
        for n, v in enumerate(dims):
            d.dims[n] = v
        m = pkg.Model()
        if core is None:
            m.kind, m.rank = pkg.COMM_CP, rank
        else:
            m.kind = pkg.COMM_TUCKER
            for n, v in enumerate(core):
                m.core_dims[n] = v
        o = pkg._opts(beta, 1e-12, None, 1, False)
        return lib.comm_workspace_bytes(ctypes.byref(d), ctypes.byref(m), ctypes.byref(o), op)

    three = ws((5600, 60, 50), rank=10)
    four = ws((80, 70, 60, 50), rank=10)
    assert three > 0 and four > three  # the view's buffers plus the grouped modes'
    assert ws((6, 5, 7, 30, 40), rank=4, beta=1.5) > 0
    assert ws((80, 70, 60, 50), core=(10, 9, 8, 7)) > ws((80, 70, 60), core=(10, 9, 8))
    assert ws((27, 24, 7, 100, 100), core=(10, 10, 5, 10, 10)) > 0
    assert ws((400, 300, 200, 2, 3), core=(2, 2, 2, 2, 2)) == 0  # I_1 ... I_4 > 2^24
    assert ws((80, 70, 60, 50), core=(10, 9, 8, 33)) == 0
    assert ws((80, 70, 60), core=(10, 9, 8)) > 0
    assert ws((4096, 4097, 2, 2), rank=4) == 0
    assert ws((40, 50), rank=4) == 0


def test_cache_option_values():
    import paper_2602_14683_amd as pkg
    header = open(HEADER).read()
    assert int(re.search(r"#define COMM_CACHE_AUTO \((-?\d+)\)", header).group(1)) == pkg.COMM_CACHE_AUTO
    assert pkg._opts(0.5, 1e-12, None, cache_pq="auto").cache_pq == pkg.COMM_CACHE_AUTO
    assert pkg._opts(0.5, 1e-12, None, cache_pq=True).cache_pq == 1
    assert pkg._opts(0.5, 1e-12, None, cache_pq=False).cache_pq == 0
    with pytest.raises(ValueError):
        pkg._opts(0.5, 1e-12, None, cache_pq="always")
