"""Host-side tests of the C ABI: the library loads, exports every declared symbol,
and validates shapes and options without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1905_05559_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return L.load()
    except ImportError as e:  # the library is built by __graft_entry__.build()
        pytest.skip(str(e))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(hess_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = _lib()
    declared = _declared_functions()
    assert set(declared) == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _mlp(T, acts=None, dtype=1):
    T_ = (C.c_int64 * len(T))(*T)
    acts = acts if acts is not None else [0] * (len(T) - 2)
    A_ = (C.c_int32 * max(1, len(acts)))(*acts)
    m = L.HessMlp(len(T), T_, A_, dtype, None, None)
    m._keep = (T_, A_)
    return m


def test_num_params_and_errors():
    lib = _lib()
    P = C.c_int64()
    assert lib.hess_num_params(C.byref(_mlp([784, 100, 10])), C.byref(P)) == 0 and P.value == 79510
    assert lib.hess_num_params(C.byref(_mlp([64, 64, 10])), C.byref(P)) == 0 and P.value == 4810
    assert lib.hess_num_params(C.byref(_mlp([4, 8, 3])), C.byref(P)) == 0 and P.value == 67
    assert lib.hess_num_params(C.byref(_mlp([64, 32])), C.byref(P)) == 0 and P.value == 2080
    assert lib.hess_num_params(C.byref(_mlp([5])), C.byref(P)) == 2          # L < 2
    assert lib.hess_num_params(C.byref(_mlp([5, 0, 3])), C.byref(P)) == 2    # zero width
    assert lib.hess_num_params(C.byref(_mlp([5, 4, 3], acts=[7])), C.byref(P)) == 1  # bad act
    assert lib.hess_num_params(C.byref(_mlp([5, 4, 3], dtype=9)), C.byref(P)) == 1   # bad dtype
    assert lib.hess_num_params(C.byref(_mlp([1 << 20, 1 << 20, 3])), C.byref(P)) == 2  # P overflow
    assert lib.hess_num_params(None, C.byref(P)) == 1


def test_workspace_sizes_are_positive_and_monotone():
    lib = _lib()
    m = _mlp([64, 64, 10], [1])
    sizes = {}
    for op in ("exact", "opg"):
        for prec in ("f64", "f32"):
            for N in (100, 10000):
                d = L.HessData(N, 1, None, None)
                nb = C.c_size_t()
                assert lib.hess_workspace_size(None, L.OP[op], C.byref(m), C.byref(d), L.PREC[prec], 0, None,
                                               C.byref(nb)) == 0
                sizes[(op, prec, N)] = nb.value
    for op in ("exact", "opg"):
        for prec in ("f64", "f32"):
            assert 0 < sizes[(op, prec, 100)] < sizes[(op, prec, 10000)]
    bad = L.HessData(0, 1, None, None)
    nb = C.c_size_t()
    assert lib.hess_workspace_size(None, 0, C.byref(m), C.byref(bad), 1, 0, None, C.byref(nb)) == 2


def test_exact_cols_workspace_and_errors():
    lib = _lib()
    m = _mlp([64, 64, 10], [1])
    d = L.HessData(1000, 1, None, None)
    sizes = []
    for ncols in (1, 100, 512, 513, 4000):
        nb = C.c_size_t()
        assert lib.hess_workspace_size(None, L.OP["exact_cols"], C.byref(m), C.byref(d), L.PREC["f32"], ncols,
                                       None, C.byref(nb)) == 0
        sizes.append(nb.value)
    # blocks of at most 512 columns: the workspace stops growing past one block
    assert sizes[0] < sizes[1] < sizes[2] == sizes[3] == sizes[4]
    nb = C.c_size_t()
    assert lib.hess_workspace_size(None, L.OP["exact_cols"], C.byref(m), C.byref(d), L.PREC["f32"], 0, None,
                                   C.byref(nb)) == 2  # HESS_E_SHAPE
    assert lib.hess_workspace_size(None, L.OP["exact_cols"], C.byref(m), C.byref(d), L.PREC["bf16"], 10, None,
                                   C.byref(nb)) == 10  # HESS_E_UNSUPPORTED


def test_status_strings():
    lib = _lib()
    for code in L.STATUS_NAMES:
        assert len(lib.hess_status_str(code)) > 0
