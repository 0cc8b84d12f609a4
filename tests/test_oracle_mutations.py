"""The oracle's pins catch plausible mistakes (CPU only).

Each test plants one mistake in a copy of the oracle -- a dropped term, a
wrong comparison, a missing exclusion, a wrong monoid rule -- and checks that
the brute-force pin used by tests/test_oracle.py rejects the mutant.  This is
what makes the pins worth trusting: a pin that cannot tell a broken oracle
from the real one proves nothing.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import importlib.util

from oracle import brute
from paper_1609_07008_amd import graphgen as gg

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
ORACLE_C = os.path.join(ORACLE_DIR, "brandes.c")
FRONTIER_PY = os.path.join(ORACLE_DIR, "frontier.py")

GRAPHS = [gg.random_small_graph(8, 0.45, 4, (1, 2)), gg.random_small_graph(9, 0.4, 5, None),
          gg.random_small_graph(10, 0.3, 7, (1, 5))]


def brute_ref(g):
    per, lam = brute.brute_bc(g, range(g.n))
    dist = np.array([[(-1 if t is None else t) for t in p["tau"]] for p in per])
    sigma = np.array([[float(x) for x in p["sigma"]] for p in per])
    delta = np.array([[float(x) for x in p["delta"]] for p in per])
    return dist, sigma, delta, np.array([float(x) for x in lam])


def agrees(g, dist, sigma, delta, lam):
    d0, s0, de0, l0 = brute_ref(g)
    return (np.array_equal(dist, d0) and np.allclose(sigma, s0, rtol=1e-12, atol=0)
            and np.allclose(delta, de0, rtol=1e-12, atol=1e-14)
            and np.allclose(lam, l0, rtol=1e-12, atol=1e-14))


def build_mutant(tmp_path, old, new):
    src = open(ORACLE_C).read()
    assert old in src, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(path)],
                   check=True, capture_output=True)
    return ctypes.CDLL(str(lib))


def run_c(lib, g):
    n = g.n
    P = ctypes.c_void_p
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    col = np.ascontiguousarray(g.col, np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, np.int32)
    src = np.arange(n, dtype=np.int32)
    lam = np.zeros(n)
    dist = np.empty((n, n), np.int64)
    sigma = np.empty((n, n))
    delta = np.empty((n, n))
    height = np.empty((n, n), np.int32)
    f = lib.oracle_bc
    f.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int32]
    f.restype = ctypes.c_int
    rc = f(n, rp.ctypes.data_as(P), col.ctypes.data_as(P),
           None if w is None else w.ctypes.data_as(P), src.ctypes.data_as(P), n,
           lam.ctypes.data_as(P), dist.ctypes.data_as(P), sigma.ctypes.data_as(P),
           delta.ctypes.data_as(P), height.ctypes.data_as(P), 1)
    assert rc == 0
    return dist, sigma, delta, lam


C_MUTATIONS = {
    "dependency drops the 1": ("(1.0 + k->delta[x])", "(k->delta[x])"),
    "relaxation uses <=": ("if (nd < k->dist[x]) {", "if (nd <= k->dist[x]) {"),
    "source not excluded": ("if (v != s) my[v] += k.delta[v];", "my[v] += k.delta[v];"),
    "bfs overwrites counts": ("if (k->dist[x] == dn) k->sigma[x] += k->sigma[v];",
                              "if (k->dist[x] == dn) k->sigma[x] = k->sigma[v];"),
    "ties not counted": ("} else if (nd == k->dist[x]) {\n                    k->sigma[x] += k->sigma[v];",
                         "} else if (nd == k->dist[x]) {\n                    k->sigma[x] += 0.0;"),
    "successor test off by one": ("k->dist[v] + wt == k->dist[x]", "k->dist[v] + wt + 1 == k->dist[x]"),
}


def test_unmutated_c_oracle_agrees(tmp_path):
    lib = build_mutant(tmp_path, "int oracle_max_threads", "int oracle_max_threads")
    for g in GRAPHS:
        assert agrees(g, *run_c(lib, g))


@pytest.mark.parametrize("name", sorted(C_MUTATIONS))
def test_c_oracle_mutants_are_caught(tmp_path, name):
    old, new = C_MUTATIONS[name]
    lib = build_mutant(tmp_path, old, new)
    assert not all(agrees(g, *run_c(lib, g)) for g in GRAPHS), f"pin missed mutant: {name}"


def frontier_pin_holds(mod) -> bool:
    """The pin of tests/test_oracle.py: frontiers against enumerated walks."""
    graphs = [gg.random_small_graph(8, 0.45, 4, (1, 3)), gg.random_small_graph(9, 0.4, 5, None),
              gg.directed_rmat_graph(3, 4, 4, wrange=(1, 3))]
    for g in graphs:
        for s in range(g.n):
            fr = mod.forward_frontiers(g, s)
            ell, _ = brute.walk_minima(g, s, len(fr))
            best = [ell[0][v] for v in range(g.n)]
            for j in range(1, len(fr) + 1):
                want = [ell[j][v] is not None and (best[v] is None or ell[j][v] <= best[v])
                        for v in range(g.n)]
                if fr[j - 1].tolist() != want:
                    return False
                best = [b if e is None else (e if b is None else min(b, e))
                        for b, e in zip(best, ell[j])]
            if fr[-1].any():
                return False
    return True


def load_frontier_mutant(tmp_path, old, new):
    src = open(FRONTIER_PY).read()
    assert old in src, old
    path = tmp_path / "frontier_mutant.py"
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location("frontier_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


FRONTIER_MUTATIONS = {
    "ties with shorter walks dropped": ("F = (nxt < INF) & (nxt <= L)", "F = (nxt < INF) & (nxt < L)"),
    "no comparison with shorter walks": ("F = (nxt < INF) & (nxt <= L)", "F = (nxt < INF)"),
    "L never lowered": ("        L = np.minimum(L, nxt)\n        ell = nxt\n        if not F.any():\n            return out",
                        "        ell = nxt\n        if not F.any():\n            return out"),
    "arcs taken head to tail": ("order = np.argsort(v, kind=\"stable\")", "order = np.argsort(u, kind=\"stable\")"),
    "weights dropped": ("cand = ell[self.tail] + self.weight", "cand = ell[self.tail] + 1"),
    "max instead of min": ("np.minimum.reduceat(cand, self.starts)", "np.maximum.reduceat(cand, self.starts)"),
}


def test_unmutated_frontier_oracle_agrees(tmp_path):
    assert frontier_pin_holds(load_frontier_mutant(tmp_path, "INF = ", "INF = "))


@pytest.mark.parametrize("name", sorted(FRONTIER_MUTATIONS))
def test_frontier_mutants_are_caught(tmp_path, name):
    old, new = FRONTIER_MUTATIONS[name]
    mod = load_frontier_mutant(tmp_path, old, new)
    try:
        ok = frontier_pin_holds(mod)
    except Exception:
        ok = False          # a mutant that crashes or never empties is caught too
    assert not ok, f"pin missed mutant: {name}"


def fixpoint_pin_holds(mod) -> bool:
    """The pins of tests/test_oracle.py for the widest and reciprocal-sum
    fixpoints: values against simple paths, product counts against walks."""
    f32 = np.float32
    for g in (gg.random_small_graph(8, 0.45, 4, (1, 3)), gg.random_small_graph(7, 0.5, 11, (1, 9))):
        for s in range(g.n):
            wide = [0] * g.n
            res = [f32(np.inf)] * g.n
            for path, ws in brute.simple_path_arcs(g, s):
                x = f32(0.0)
                for w in ws:
                    x = f32(x + f32(f32(1.0) / f32(w)))
                wide[path[-1]] = max(wide[path[-1]], min(ws) if ws else int(mod.WIDE_INF))
                res[path[-1]] = min(res[path[-1]], x)
            L, kw = mod.fixpoint(g, s, "widest")
            R, kr = mod.fixpoint(g, s, "resist")
            if L.tolist() != wide or [float(x) for x in R] != [float(x) for x in res]:
                return False
            for op, k, fold, better, start in (
                    ("widest", kw, lambda a, w: min(a, w), lambda a, b: a > b, int(mod.WIDE_INF)),
                    ("resist", kr, lambda a, w: f32(a + f32(f32(1.0) / f32(w))), lambda a, b: a < b, f32(0.0))):
                ell = brute.walk_best(g, s, g.n + 1, fold, better, start)
                best = list(ell[0])
                expect = None
                for j in range(1, g.n + 2):
                    up = [v for v in range(g.n) if ell[j][v] is not None
                          and (best[v] is None or better(ell[j][v], best[v]))]
                    for v in up:
                        best[v] = ell[j][v]
                    if not up:
                        expect = j
                        break
                if k != expect:
                    return False
    return True


FIXPOINT_MUTATIONS = {
    "widest takes the least candidate": ("nxt[self.has] = np.maximum.reduceat(cand, self.starts)",
                                         "nxt[self.has] = np.minimum.reduceat(cand, self.starts)"),
    "widest action adds the weight": ("cand = np.minimum(ell[self.tail], self.weight)",
                                      "cand = np.minimum(ell[self.tail] + self.weight, WIDE_INF)"),
    "widest source not unbounded": ("        ell[s] = WIDE_INF\n", "        ell[s] = 255\n"),
    "resist sums in binary64": ("recip = np.float32(1.0) / self.weight.astype(np.float32)\n            cand = ell[self.tail] + recip",
                                "recip = 1.0 / self.weight.astype(np.float64)\n            cand = ell[self.tail].astype(np.float64) + recip"),
    "resist adds the weight": ("cand = ell[self.tail] + recip", "cand = ell[self.tail] + self.weight.astype(np.float32)"),
    "ties re-enter the frontier": ("F = better(nxt, L)", "F = better(nxt, L) | ((nxt == L) & (j < 3))"),
}


def test_unmutated_fixpoint_oracle_agrees(tmp_path):
    assert fixpoint_pin_holds(load_frontier_mutant(tmp_path, "INF = ", "INF = "))


@pytest.mark.parametrize("name", sorted(FIXPOINT_MUTATIONS))
def test_fixpoint_mutants_are_caught(tmp_path, name):
    old, new = FIXPOINT_MUTATIONS[name]
    mod = load_frontier_mutant(tmp_path, old, new)
    try:
        ok = fixpoint_pin_holds(mod)
    except Exception:
        ok = False
    assert not ok, f"pin missed mutant: {name}"
