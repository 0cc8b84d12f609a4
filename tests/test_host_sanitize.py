"""The host code that runs before any device work -- CSR validation, the
transpose and renumbering, the work decomposition -- built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and fed malformed and valid
graphs.  Every array is passed in a heap block of exactly its size, so a read
past the caller's arrays (or any undefined behaviour) aborts the harness;
each malformed graph must be rejected with the right status and a message."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1609_07008_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_07008_amd", "csrc")
EINVAL, EOVERFLOW = -1, -4


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no g++ or ROCm headers")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_check")
    r = subprocess.run([cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                        "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "sanitize_check.cpp"),
                        os.path.join(CSRC, "order.cpp"), os.path.join(CSRC, "graph.cpp"),
                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in (r.stderr or ""):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def encode(n, rp, col, w=None, undirected=True) -> bytes:
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col, np.int32)
    parts = [np.array([n], np.int32).tobytes(), np.array([col.size], np.int64).tobytes(),
             np.array([w is not None, undirected], np.int32).tobytes(), rp.tobytes(), col.tobytes()]
    if w is not None:
        parts.append(np.asarray(w, np.int32).tobytes())
    return b"".join(parts)


def run(harness, tmp_path, cases):
    src, dst = str(tmp_path / "cases.bin"), str(tmp_path / "out.bin")
    with open(src, "wb") as f:
        for c in cases:
            f.write(encode(**c))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([harness, src, dst], capture_output=True, text=True, env=env)
    assert r.returncode == 0, f"harness failed ({r.returncode}):\n{r.stderr[-3000:]}"
    return np.fromfile(dst, dtype=np.int32).reshape(-1, 6)


MALFORMED = [
    (dict(n=0, rp=[0], col=[]), EINVAL),                                    # no vertices
    (dict(n=2, rp=[0, 1, 2], col=[1, 0], w=[1, 0]), EINVAL),                # zero weight
    (dict(n=2, rp=[0, 1, 2], col=[1, 0], w=[-3, -3]), EINVAL),              # negative weight
    (dict(n=2, rp=[0, 1, 2], col=[0, 1]), EINVAL),                          # self-loops
    (dict(n=3, rp=[0, 2, 3, 4], col=[1, 1, 0, 0]), EINVAL),                 # duplicate arc
    (dict(n=2, rp=[0, 1, 2], col=[5, 0]), EINVAL),                          # column out of range
    (dict(n=2, rp=[0, 1, 2], col=[-1, 0]), EINVAL),                         # negative column
    (dict(n=2, rp=[1, 1, 2], col=[1, 0]), EINVAL),                          # row_ptr[0] != 0
    (dict(n=3, rp=[0, 2, 1, 2], col=[1, 2]), EINVAL),                       # decreasing row_ptr
    (dict(n=2, rp=[0, 9, 2], col=[1, 0]), EINVAL),                          # row past the arcs
    (dict(n=2, rp=[0, 1, 3], col=[1, 0]), EINVAL),                          # row_ptr[n] != n_arcs
    (dict(n=3, rp=[0, 2, 3, 4], col=[2, 1, 0, 0]), EINVAL),                 # unsorted row
    (dict(n=20000, rp=[0, 1, 2] + [2] * 19998, col=[1, 0], w=[200000, 200000]), EOVERFLOW),
]


def test_malformed_graphs_are_rejected_without_stray_reads(harness, tmp_path):
    res = run(harness, tmp_path, [c for c, _ in MALFORMED])
    assert res[:, 0].tolist() == [code for _, code in MALFORMED]


def test_valid_graphs_pass_every_host_step(harness, tmp_path):
    graphs = [gg.path_graph(1), gg.path_graph(2), gg.star_graph(3000), gg.grid_graph(7, 9),
              gg.er_graph(500, 6, 3, (1, 100)), gg.rmat_graph(10, 8, 5),
              gg.csr_from_edges(6, [], [], None, "no_arcs")]
    cases = [dict(n=g.n, rp=g.row_ptr, col=g.col, w=g.w) for g in graphs]
    asym = gg.csr_from_edges(3, [0, 1], [1, 2], None)
    cases.append(dict(n=3, rp=[0, 1, 2, 2], col=[1, 2], undirected=False))   # a directed path
    d = gg.directed_rmat_graph(8, 4, 2, wrange=(1, 9))
    cases.append(dict(n=d.n, rp=d.row_ptr, col=d.col, w=d.w, undirected=False))
    res = run(harness, tmp_path, cases)
    assert np.all(res[:, 0] == 0)
    assert res[:-2, 2].tolist() == [1] * (len(graphs))          # undirected inputs are symmetric
    assert res[-2, 2] == 0                                       # the directed path is not
    assert res[graphs.index(graphs[4]), 1] == graphs[4].w.max()
    assert res[2, 4] > 0                                         # the star's hub row is split
    del asym


def test_sanitizer_catches_a_planted_stray_read(tmp_path):
    """The harness is only worth its pass if a read one past the caller's
    column array aborts it: plant one in a copy of order.cpp (on the CPU)."""
    cxx = shutil.which("g++")
    if not cxx or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no g++ or ROCm headers")
    src = open(os.path.join(CSRC, "order.cpp")).read()
    old = "const int32_t c = col[e];"
    assert old in src
    mutant = tmp_path / "order.cpp"
    stray = "const int32_t c = col[e]; (void)((const volatile int32_t *)col)[e + 1];"
    mutant.write_text(src.replace(old, stray, 1)
                      .replace('#include "../../include/mfbc.h"', '#include "mfbc.h"'))
    exe = str(tmp_path / "mutant_check")
    r = subprocess.run([cxx, "-O0", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
                        "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "sanitize_check.cpp"), str(mutant),
                        os.path.join(CSRC, "graph.cpp"), "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in (r.stderr or ""):
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr
    g = gg.path_graph(5)
    with open(tmp_path / "c.bin", "wb") as f:
        f.write(encode(n=g.n, rp=g.row_ptr, col=g.col))
    r = subprocess.run([exe, str(tmp_path / "c.bin"), str(tmp_path / "o.bin")],
                       capture_output=True, text=True)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
