"""Host-side work decomposition of the library (``csrc/graph.cpp``), built
with g++ and checked on the CPU against the properties the kernels rely on:
the tasks tile every arc exactly once in CSR order; a light run holds 1..64
whole rows of degree <= heavy, at most run_verts of them, and stays within
run_arcs unless it is a single row; every heavier row is one hub cut into
consecutive slices of at most `slice` arcs whose partial slots are
numbered consecutively; and every vertex belongs to exactly one task or hub."""
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
    if not cxx or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no g++ or ROCm headers")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    subprocess.run([cxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
                    os.path.join(CSRC, "graph.cpp"), "-o", exe], check=True)
    return exe


def plan(harness, tmp_path, rp, params):
    rp = np.asarray(rp, np.int64)
    n = rp.size - 1
    src, dst = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(src, "wb") as f:
        np.array([n, *params], np.int32).tofile(f)
        rp.tofile(f)
    subprocess.run([harness, src, dst], check=True)
    raw = open(dst, "rb").read()
    head = np.frombuffer(raw, np.int32, 5)
    nt, nh = int(head[2]), int(head[3])
    rec = np.dtype([("v0", "<i4"), ("v1", "<i4"), ("hub", "<i4"), ("part", "<i4"),
                    ("e0", "<i8"), ("e1", "<i8")])
    tasks = np.frombuffer(raw, rec, nt, 20)
    hubs = np.frombuffer(raw, np.int32, 3 * nh, 20 + rec.itemsize * nt).reshape(nh, 3)
    return head, tasks, hubs


def check(rp, params, head, tasks, hubs):
    run_arcs, run_verts, heavy, slice_ = params
    rp = np.asarray(rp, np.int64)
    n, deg = rp.size - 1, np.diff(rp)
    # arcs tiled exactly once, in order
    assert tasks["e0"][0] == 0 and tasks["e1"][-1] == rp[-1]
    assert np.array_equal(tasks["e0"][1:], tasks["e1"][:-1])
    assert np.all(tasks["e1"] >= tasks["e0"])
    covered = np.zeros(n, np.int64)
    slots = 0
    for h, (v, first, nparts) in enumerate(hubs):
        assert deg[v] > heavy
        assert nparts == -(-deg[v] // slice_)
        assert first == slots
        slots += nparts
        mine = tasks[tasks["hub"] == h]
        assert len(mine) == nparts
        assert np.all(mine["v0"] == v) and np.all(mine["v1"] == v + 1)
        assert np.array_equal(mine["part"], first + np.arange(nparts))
        assert mine["e0"][0] == rp[v] and mine["e1"][-1] == rp[v + 1]
        assert np.all(mine["e1"] - mine["e0"] <= slice_) and np.all(mine["e1"] > mine["e0"])
        covered[v] += 1
    assert slots == head[4]
    light = tasks[tasks["hub"] < 0]
    assert np.all(light["part"] == -1)
    for t in light:
        rows = np.arange(t["v0"], t["v1"])
        assert 1 <= rows.size <= min(max(run_verts, 1), 64)
        assert np.all(deg[rows] <= heavy)
        assert t["e0"] == rp[t["v0"]] and t["e1"] == rp[t["v1"]]
        assert rows.size == 1 or t["e1"] - t["e0"] <= run_arcs
        covered[rows] += 1
    assert np.all(covered == 1)
    # default parameters stay in the ranges the kernels accept
    assert 64 <= head[0] <= 512 and 1 <= head[1] <= 64


GRAPHS = {
    "rmat12": gg.rmat_graph(12, 16, 3),
    "star3000": gg.star_graph(3000),
    "er500_k40": gg.er_graph(500, 40, 5),
    "path100": gg.path_graph(100),
}
PARAMS = [(512, 64, 1024, 512), (64, 1, 100, 17), (1, 64, 2, 1), (700, 3, 40, 7), (4096, 64, 10 ** 6, 512)]


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("params", PARAMS)
def test_tasks_tile_the_arcs(harness, tmp_path, name, params):
    rp = GRAPHS[name].row_ptr
    head, tasks, hubs = plan(harness, tmp_path, rp, params)
    check(rp, params, head, tasks, hubs)


def test_isolated_and_empty_rows(harness, tmp_path):
    """Zero-degree rows join light runs (an empty run is still one task)."""
    rp = np.array([0, 0, 0, 3, 3, 3, 10, 10], np.int64)
    params = (2, 4, 5, 3)
    head, tasks, hubs = plan(harness, tmp_path, rp, params)
    check(rp, params, head, tasks, hubs)
    assert len(hubs) == 1 and hubs[0][0] == 5
