"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point include/mfbc.h declares, and rejects malformed graphs before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_07008_amd import mfbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mfbc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfbc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mfbc.load_library()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    from paper_1609_07008_amd import serve
    assert set(names) == set(mfbc.SIGNATURES) | set(serve.SERVER_SIGNATURES)


def test_library_is_built_for_gfx950():
    data = open(mfbc.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _load(n, rp, col, w=None, flags=mfbc.MFBC_UNDIRECTED):
    lib = mfbc.load_library()
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.int32)
        wp = w.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    rc = lib.mfbc_load_graph(n, int(col.size), rp.ctypes.data_as(ctypes.c_void_p),
                             col.ctypes.data_as(ctypes.c_void_p), wp, flags, None,
                             ctypes.byref(h))
    return rc, lib.mfbc_last_error().decode()


@pytest.mark.parametrize("case", [
    dict(n=0, rp=[0], col=[]),                                        # no vertices
    dict(n=2, rp=[0, 1, 2], col=[1, 0], w=[1, 0]),                    # zero weight
    dict(n=2, rp=[0, 1, 2], col=[1, 0], w=[-3, -3]),                  # negative weight
    dict(n=2, rp=[0, 1, 1], col=[1]),                                 # asymmetric undirected
    dict(n=2, rp=[0, 1, 2], col=[1, 0], w=[2, 3]),                    # unequal weights
    dict(n=2, rp=[0, 1, 2], col=[0, 1]),                              # self-loops
    dict(n=3, rp=[0, 2, 3, 4], col=[1, 1, 0, 0]),                     # duplicate arc
    dict(n=2, rp=[0, 1, 2], col=[5, 0]),                              # column out of range
    dict(n=2, rp=[1, 1, 2], col=[1, 0]),                              # row_ptr[0] != 0
    dict(n=3, rp=[0, 2, 1, 2], col=[1, 2]),                           # decreasing row_ptr
    dict(n=2, rp=[0, 1, 2], col=[1, 0], flags=7),                     # bad flags
])
def test_invalid_graphs_are_rejected_on_the_host(case):
    rc, msg = _load(case["n"], case["rp"], case["col"], case.get("w"),
                    case.get("flags", mfbc.MFBC_UNDIRECTED))
    assert rc == mfbc.MFBC_EINVAL, (rc, msg)
    assert msg


def test_distance_overflow_is_rejected():
    n = 20000
    rp = [0, 1, 2] + [2] * (n - 2)
    rc, msg = _load(n, rp, [1, 0], [200000, 200000])
    assert rc == mfbc.MFBC_EOVERFLOW, (rc, msg)


def test_free_null_is_ok():
    assert mfbc.load_library().mfbc_free_graph(None) == 0


def test_null_handles_are_rejected_before_device_work():
    """Every entry point that takes a graph or server handle answers a NULL one
    with EINVAL and a message before any device call (so this runs without a
    GPU); the two release calls accept NULL."""
    from paper_1609_07008_amd import serve
    lib = mfbc.load_library()
    for name, (args, res) in serve.SERVER_SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    sigs = {**mfbc.SIGNATURES, **serve.SERVER_SIGNATURES}
    ints = (ctypes.c_int, ctypes.c_long, ctypes.c_uint, ctypes.c_int64, ctypes.c_int32)
    checked = 0
    for name, (args, _) in sigs.items():
        if name in ("mfbc_last_error", "mfbc_load_graph", "mfbc_bc_many"):
            continue
        call = [0 if a in ints else None for a in args]
        rc = getattr(lib, name)(*call)
        if name in ("mfbc_free_graph", "mfbc_server_free"):
            assert rc == mfbc.MFBC_OK, name
            continue
        assert rc == mfbc.MFBC_EINVAL, (name, rc)
        assert lib.mfbc_last_error(), name
        checked += 1
    assert checked >= 20
    # the calls without a leading handle: no output slot, no graph array
    assert lib.mfbc_load_graph(2, 2, None, None, None, mfbc.MFBC_UNDIRECTED, None, None) == mfbc.MFBC_EINVAL
    assert lib.mfbc_bc_many(1, None, None, None, None, None, None, None) == mfbc.MFBC_EINVAL
    assert lib.mfbc_bc_many(-1, None, None, None, None, None, None, None) == mfbc.MFBC_EINVAL
    assert lib.mfbc_bc_many(0, None, None, None, None, None, None, None) == mfbc.MFBC_OK
