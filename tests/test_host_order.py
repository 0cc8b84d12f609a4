"""Host-side CSR reorganisation of the library (``csrc/order.cpp``), built
with g++ and checked on the CPU: the descending-degree numbering (in- plus
out-degree, ties by id) and the relabelled CSRs the device copy of a graph
is built from, against an independent numpy construction (the relabelled
edge list sorted by row, then column)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1609_07008_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_07008_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("order") / "order_check")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "order_check.cpp"),
                    os.path.join(CSRC, "order.cpp"), "-o", exe], check=True)
    return exe


def run(harness, tmp_path, g, directed):
    n, arcs = g.n, int(g.row_ptr[-1])
    weighted = g.w is not None
    src, dst = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(src, "wb") as f:
        np.array([n], np.int32).tofile(f)
        np.array([arcs], np.int64).tofile(f)
        np.array([int(weighted), int(directed)], np.int32).tofile(f)
        np.asarray(g.row_ptr, np.int64).tofile(f)
        np.asarray(g.col, np.int32).tofile(f)
        if weighted:
            np.asarray(g.w, np.int32).tofile(f)
    subprocess.run([harness, src, dst], check=True)
    raw = open(dst, "rb").read()
    out, off = {}, 0

    def take(name, dtype, count):
        nonlocal off
        out[name] = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += np.dtype(dtype).itemsize * count

    take("perm", np.int32, n)
    take("rp_rev", np.int64, n + 1)
    take("col_rev", np.int32, arcs)
    if weighted:
        take("w_rev", np.int32, arcs)
    if directed:
        take("rp_out", np.int64, n + 1)
        take("col_out", np.int32, arcs)
        if weighted:
            take("w_out", np.int32, arcs)
    assert off == len(raw)
    return out


def csr_of(n, rows, cols, w):
    """CSR of an arc list, rows then columns ascending."""
    order = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols[order].astype(np.int32), None if w is None else w[order]


def expected(g):
    n = g.n
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    x = np.asarray(g.col, np.int64)
    key = np.diff(g.row_ptr) + np.bincount(x, minlength=n)       # out- plus in-degree
    iperm = np.argsort(-key, kind="stable")
    perm = np.empty(n, np.int64)
    perm[iperm] = np.arange(n)
    w = None if g.w is None else np.asarray(g.w, np.int32)
    return perm, csr_of(n, perm[x], perm[u], w), csr_of(n, perm[u], perm[x], w)


CASES = {
    "rmat9_w": (gg.rmat_graph(9, 8, 4, wrange=(1, 50)), False),
    "er300_unw": (gg.er_graph(300, 5, 7), False),
    "star50": (gg.star_graph(50), False),               # one hub, all other degrees tied
    "path40_w": (gg.path_graph(40, w=3), False),
    "directed_rmat8_w": (gg.directed_rmat_graph(8, 8, 12, wrange=(1, 9)), True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_degree_numbering_and_relabelled_csr(harness, tmp_path, name):
    g, directed = CASES[name]
    got = run(harness, tmp_path, g, directed)
    perm, rev, fwd = expected(g)
    assert np.array_equal(got["perm"], perm)
    assert np.array_equal(np.sort(got["perm"]), np.arange(g.n))
    assert np.array_equal(got["rp_rev"], rev[0])
    assert np.array_equal(got["col_rev"], rev[1])
    if g.w is not None:
        assert np.array_equal(got["w_rev"], rev[2])
    if directed:
        assert np.array_equal(got["rp_out"], fwd[0])
        assert np.array_equal(got["col_out"], fwd[1])
        if g.w is not None:
            assert np.array_equal(got["w_out"], fwd[2])
    else:
        # undirected: the reverse graph is the graph itself, renumbered
        rel = gg.relabel(g, perm)
        assert np.array_equal(got["rp_rev"], rel.row_ptr)
        assert np.array_equal(got["col_rev"], rel.col)
