"""C ABI conventions that hold without a GPU: symbols, validation before any device call."""
import ctypes

import numpy as np
import pytest

import gen


@pytest.fixture(scope="module")
def mos():
    import paper_2411_16667_amd as m

    return m


def test_every_declared_symbol_is_exported(mos):
    names = mos.exported_symbols_in_header()
    assert len(names) >= 20
    for n in names:
        assert hasattr(mos.raw, n), n


def _create(mos, n, rp, col, cost, D):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    st = mos.raw.mos_graph_create(n, col.size, D, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  cost.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  ctypes.byref(h))
    return st, h


def test_validation_precedes_device(mos):
    g, _, _ = gen.config1(0)
    # negative cost
    c = g.cost.copy(); c[10, 2] = -3
    assert _create(mos, g.n, g.row_ptr, g.col, c, 3)[0] == mos.MOS_E_NEGATIVE_COST
    # overflow risk: 2*sum + max > INT32_MAX
    c = g.cost.copy(); c[0, 0] = 2**30
    assert _create(mos, g.n, g.row_ptr, g.col, c, 3)[0] == mos.MOS_E_OVERFLOW_RISK
    # the bound is strict: 2*sum + max == INT32_MAX is refused, one less is not
    rp2 = np.array([0, 1, 2], dtype=np.int64)
    col2 = np.array([1, 0], dtype=np.int32)
    edge = np.array([[715827881], [2]], dtype=np.int32)   # 2*(a+b) + a == 2**31 - 1
    assert _create(mos, 2, rp2, col2, edge, 1)[0] == mos.MOS_E_OVERFLOW_RISK
    st, h = _create(mos, 2, rp2, col2, edge - np.array([[1], [0]], dtype=np.int32), 1)
    assert st != mos.MOS_E_OVERFLOW_RISK
    if st == mos.MOS_OK:
        mos.raw.mos_graph_destroy(h)
    # target out of range
    col = g.col.copy(); col[5] = g.n
    assert _create(mos, g.n, g.row_ptr, col, g.cost, 3)[0] == mos.MOS_E_INVALID_ARG
    # row_ptr not monotone / wrong ends
    rp = g.row_ptr.copy(); rp[3], rp[4] = rp[4], rp[3]
    assert _create(mos, g.n, rp, g.col, g.cost, 3)[0] == mos.MOS_E_INVALID_ARG
    rp = g.row_ptr.copy(); rp[-1] -= 1
    assert _create(mos, g.n, rp, g.col, g.cost, 3)[0] == mos.MOS_E_INVALID_ARG
    # D out of range
    assert _create(mos, g.n, g.row_ptr, g.col, np.zeros((g.n_arcs, 13)), 13)[0] == mos.MOS_E_INVALID_ARG
    # NULL out-parameter
    assert mos.raw.mos_graph_create(1, 0, 1, np.zeros(2, np.int64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_int64)), None, None, None) == mos.MOS_E_INVALID_ARG


def test_status_strings_and_null_handles(mos):
    for i in range(10):
        assert mos.raw.mos_status_string(i)
    assert mos.raw.mos_result_size(None) == 0
    assert mos.raw.mos_result_dim(None) == 0
    mos.raw.mos_result_destroy(None)
    mos.raw.mos_graph_destroy(None)
    mos.raw.mos_server_destroy(None)
    assert mos.raw.mos_solve(None, 0, 0, None, None) == mos.MOS_E_INVALID_ARG


def test_no_device_reported_cleanly(mos):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    g, _, _ = gen.config1(0)
    st, _ = _create(mos, g.n, g.row_ptr, g.col, g.cost, 3)
    assert st == mos.MOS_E_NO_DEVICE
    assert b"device" in mos.raw.mos_last_error()


def _header_struct_fields(name):
    """(type, field) of each member of `typedef struct { ... } name;` in mos.h,
    comments removed."""
    import re

    txt = open(__import__("paper_2411_16667_amd").HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    end = re.search(r"\}\s*" + name + r";", txt).start()
    body = txt[txt.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    return re.findall(r"(u?int(?:32|64)_t|void\s*\*|double)\s*(\w+)\s*;", body)


@pytest.mark.parametrize("name,cls", [("mos_options", "mos_options"), ("mos_stats", "mos_stats")])
def test_binding_structs_follow_the_header(mos, name, cls):
    """The ctypes mirrors of the option and statistics structs list the
    header's members in the same order with the same widths."""
    fields = _header_struct_fields(name)
    mirror = getattr(mos, cls)._fields_
    assert [f for _, f in fields] == [f for f, _ in mirror]
    width = {"int32_t": 4, "uint32_t": 4, "int64_t": 8, "uint64_t": 8, "double": 8}
    for (t, f), (_, ct) in zip(fields, mirror):
        assert ctypes.sizeof(ct) == width.get(t.replace(" ", ""), ctypes.sizeof(ctypes.c_void_p)), f


def test_status_names_follow_the_header(mos):
    """The binding's status names and values are the header's enum, in order."""
    import re

    txt = open(mos.HEADER).read()
    body = txt[txt.index("typedef enum {"):txt.index("} mos_status;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    pairs = [(n, int(v)) for n, v in re.findall(r"(MOS_[A-Z_]+)\s*=\s*(\d+)", body)]
    assert [n for n, _ in pairs] == mos.STATUS_NAMES
    assert [v for _, v in pairs] == list(range(len(pairs)))
    for n, v in pairs:
        assert getattr(mos, n) == v
        assert mos.raw.mos_status_string(v)
