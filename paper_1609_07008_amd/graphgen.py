"""Seeded synthetic inputs: graphs, source lists and request traces.

This module only *makes inputs*.  It holds none of the method's arithmetic
(no distances, path counts or centralities), so both the HIP path and the CPU
oracle may import it.  Every random draw goes through numpy's PCG64
(``numpy.random.default_rng(seed)``), so a (generator, seed) pair names one
input exactly.

Graph convention (the adjacency convention of Section 2.1): an undirected
simple graph on vertices ``0..n-1`` stored as a symmetric CSR.  Row ``v``
lists the neighbours of ``v`` in increasing order; ``w`` holds the integer
weight of each arc (both arcs of an undirected edge carry the same weight) or
is ``None`` for an unweighted graph, which means every weight is 1.  ``m`` is
the number of unique undirected edges, so the CSR has ``2*m`` arcs.

Workload shapes follow the paper's evaluation (Section 7): R-MAT power-law
graphs with quadrant probabilities (a, b, c, d) and Erdos-Renyi uniform
graphs, unweighted or with integer weights drawn uniformly from a range.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "Graph", "csr_from_edges", "er_graph", "rmat_graph", "pick_sources",
    "path_graph", "star_graph", "cycle_graph", "complete_graph",
    "complete_bipartite_graph", "grid_graph", "diamond_chain",
    "layered_bipartite", "random_small_graph", "batched_suite",
    "poisson_trace", "relabel", "scale_weights", "directed_rmat_graph",
    "DiGraph",
]


@dataclass
class Graph:
    """Undirected simple graph as a symmetric CSR (see the module docstring)."""

    n: int
    row_ptr: np.ndarray          # int64[n+1]
    col: np.ndarray              # int32[2m]
    w: Optional[np.ndarray]      # int32[2m] or None (all weights 1)
    name: str = ""

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.arcs // 2

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def max_weight(self) -> int:
        return 1 if self.w is None or self.w.size == 0 else int(self.w.max())

    def edges(self):
        """Unique undirected edges (u < v) and their weights (or None)."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degree)
        keep = rows < self.col
        w = None if self.w is None else self.w[keep]
        return rows[keep], self.col[keep].astype(np.int64), w

    def weights_or_ones(self) -> np.ndarray:
        if self.w is None:
            return np.ones(self.arcs, dtype=np.int32)
        return self.w


def csr_from_edges(n: int, u, v, w=None, name: str = "") -> Graph:
    """Symmetric CSR from unique undirected edges (u[i], v[i]), u != v.

    The caller guarantees uniqueness and the absence of self-loops; the
    result's rows are sorted by neighbour id.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n) if src.size else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    ww = None
    if w is not None:
        w = np.asarray(w, dtype=np.int32)
        ww = np.concatenate([w, w])[order].astype(np.int32)
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), w=ww, name=name)


def _dedupe_undirected(n: int, a: np.ndarray, b: np.ndarray):
    """Drop self-loops and duplicate undirected pairs; return sorted (lo, hi)."""
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    keep = lo != hi
    key = np.unique(lo[keep] * np.int64(n) + hi[keep])
    return key // n, key % n


def _draw_weights(rng, count: int, wrange):
    if wrange is None:
        return None
    lo, hi = int(wrange[0]), int(wrange[1])
    if lo < 1 or hi < lo:
        raise ValueError("weights must be integers >= 1")
    return rng.integers(lo, hi + 1, size=count, dtype=np.int64).astype(np.int32)


def relabel(g: Graph, perm: np.ndarray, name: str = "") -> Graph:
    """The same graph with vertex ``i`` renamed ``perm[i]``."""
    perm = np.asarray(perm, dtype=np.int64)
    u, v, w = g.edges()
    return csr_from_edges(g.n, perm[u], perm[v], w, name or g.name)


def scale_weights(g: Graph, factor: int) -> Graph:
    """The same graph with every weight multiplied by ``factor``."""
    w = g.weights_or_ones().astype(np.int64) * int(factor)
    return Graph(g.n, g.row_ptr.copy(), g.col.copy(), w.astype(np.int32), g.name)


def er_graph(n: int, k: float, seed: int, wrange=None, name: str = "") -> Graph:
    """Erdos-Renyi G(n, M) with M = round(n*k/2) unique undirected edges.

    Pairs are drawn uniformly, de-duplicated, and M of the distinct pairs are
    kept uniformly at random, which yields a uniform M-subset of all pairs.
    Weights (if ``wrange``) are drawn per undirected edge.
    """
    rng = np.random.default_rng(seed)
    M = int(round(n * k / 2))
    total = n * (n - 1) // 2
    if M > total:
        raise ValueError("too many edges for n")
    lo = np.empty(0, np.int64)
    hi = np.empty(0, np.int64)
    while lo.size < M:
        draw = int((M - lo.size) * 1.2) + 16
        a = rng.integers(0, n, size=draw, dtype=np.int64)
        b = rng.integers(0, n, size=draw, dtype=np.int64)
        l2, h2 = _dedupe_undirected(n, np.concatenate([lo, a]), np.concatenate([hi, b]))
        lo, hi = l2, h2
    pick = np.sort(rng.choice(lo.size, size=M, replace=False))
    lo, hi = lo[pick], hi[pick]
    w = _draw_weights(rng, M, wrange)
    return csr_from_edges(n, lo, hi, w, name or f"er_n{n}_k{k:g}_s{seed}")


def _rmat_pairs(rng, scale: int, count: int, abcd):
    a, b, c, _ = abcd
    u = np.zeros(count, dtype=np.int64)
    v = np.zeros(count, dtype=np.int64)
    for _ in range(scale):
        r = rng.random(count)
        # quadrant a: (0,0); b: (0,1); c: (1,0); d: (1,1)
        ubit = r >= a + b
        vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
        u = (u << 1) | ubit
        v = (v << 1) | vbit
    return u, v


def rmat_graph(scale: int, ef: int, seed: int, abcd=(0.57, 0.19, 0.19, 0.05),
               wrange=None, relabel_ids: bool = True, n: Optional[int] = None,
               name: str = "") -> Graph:
    """R-MAT graph: ``ef * 2**scale`` pairs, symmetrised, loops and duplicates dropped.

    With ``relabel_ids`` the vertex ids are permuted at random (after the
    de-duplication), so hubs are not clustered at low ids.  With ``n`` smaller
    than ``2**scale`` pairs with an endpoint >= n are rejected (used for graphs
    whose size is not a power of two).  Weights are drawn per undirected edge.
    """
    rng = np.random.default_rng(seed)
    N = 1 << scale
    nv = N if n is None else int(n)
    u, v = _rmat_pairs(rng, scale, ef * nv if n is not None else ef * N, abcd)
    if n is not None:
        keep = (u < nv) & (v < nv)
        u, v = u[keep], v[keep]
    lo, hi = _dedupe_undirected(nv, u, v)
    if relabel_ids:
        perm = rng.permutation(nv).astype(np.int64)
        lo, hi = perm[lo], perm[hi]
        a2 = np.minimum(lo, hi)
        b2 = np.maximum(lo, hi)
        key = np.sort(a2 * np.int64(nv) + b2)
        lo, hi = key // nv, key % nv
    w = _draw_weights(rng, lo.size, wrange)
    return csr_from_edges(nv, lo, hi, w, name or f"rmat_s{scale}_ef{ef}_s{seed}")


def pick_sources(g: Graph, count: int, seed: int, replace: bool = False) -> np.ndarray:
    """``count`` source vertices of degree >= 1, drawn without replacement."""
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(g.degree > 0)
    if not replace and count > cand.size:
        raise ValueError("not enough non-isolated vertices")
    return rng.choice(cand, size=count, replace=replace).astype(np.int32)


# ---------------------------------------------------------------- small families
def path_graph(n: int, w=None) -> Graph:
    u = np.arange(n - 1)
    return csr_from_edges(n, u, u + 1, None if w is None else np.full(n - 1, w), f"path{n}")


def star_graph(k: int) -> Graph:
    """Centre 0 joined to leaves 1..k."""
    return csr_from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1), None, f"star{k}")


def cycle_graph(n: int) -> Graph:
    u = np.arange(n)
    return csr_from_edges(n, u, (u + 1) % n, None, f"cycle{n}")


def complete_graph(n: int, w=None) -> Graph:
    iu = np.triu_indices(n, 1)
    ww = None if w is None else np.full(iu[0].size, w)
    return csr_from_edges(n, iu[0], iu[1], ww, f"K{n}")


def complete_bipartite_graph(a: int, b: int) -> Graph:
    """Side A = 0..a-1, side B = a..a+b-1."""
    uu, vv = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return csr_from_edges(a + b, uu.ravel(), vv.ravel(), None, f"K{a},{b}")


def grid_graph(a: int, b: int) -> Graph:
    """a x b grid; vertex (i, j) has id i*b + j."""
    ids = np.arange(a * b).reshape(a, b)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return csr_from_edges(a * b, u, v, None, f"grid{a}x{b}")


def diamond_chain(k: int) -> Graph:
    """k diamonds in series: hub 0, then (top, bottom, joint) per diamond.

    Hubs are 0, 3, 6, ..., 3k; diamond i joins hub 3i to hub 3i+3 through two
    middle vertices 3i+1 and 3i+2.
    """
    u, v = [], []
    for i in range(k):
        h, t, b, j = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        u += [h, h, t, b]
        v += [t, b, j, j]
    return csr_from_edges(3 * k + 1, u, v, None, f"diamonds{k}")


def layered_bipartite(L: int, width: int) -> Graph:
    """Vertex 0, then L layers of ``width`` vertices, consecutive layers fully joined."""
    n = 1 + L * width
    u, v = [], []
    prev = [0]
    for layer in range(L):
        cur = list(range(1 + layer * width, 1 + (layer + 1) * width))
        for a in prev:
            for b in cur:
                u.append(a)
                v.append(b)
        prev = cur
    return csr_from_edges(n, u, v, None, f"layers{L}x{width}")


def random_small_graph(n: int, p: float, seed: int, wrange=None) -> Graph:
    """G(n, p) on a handful of vertices (for brute-force pins)."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < p
    lo, hi = iu[0][keep], iu[1][keep]
    w = _draw_weights(rng, lo.size, wrange)
    return csr_from_edges(n, lo, hi, w, f"gnp{n}_{p:g}_s{seed}")


# ---------------------------------------------------------------- workload suites
def batched_specs(count: int = 256, seed0: int = 1000, nmin: int = 200,
                  nmax: int = 20000, kmin: float = 4, kmax: float = 64) -> list:
    """(kind, n, average degree, sub-seed) of every graph of ``batched_suite``.

    Graph ``g`` is drawn from seed ``seed0 + g``: its kind is ER or R-MAT with
    probability 1/2, n is log-uniform in [nmin, nmax], the average degree is
    uniform in [kmin, kmax].
    """
    out = []
    for gi in range(count):
        rng = np.random.default_rng(seed0 + gi)
        kind = "er" if rng.random() < 0.5 else "rmat"
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        k = float(rng.uniform(kmin, kmax))
        sub = int(rng.integers(0, 2**31 - 1))
        out.append((kind, n, k, sub))
    return out


def batched_graph(gi: int, spec, wrange=(1, 100)) -> Graph:
    """Graph ``gi`` of the batched suite from its spec (see batched_specs).
    R-MAT graphs use scale ceil(log2 n) and reject endpoints >= n."""
    kind, n, k, sub = spec
    if kind == "er":
        return er_graph(n, k, sub, wrange, name=f"batch{gi}_er_n{n}")
    scale = int(np.ceil(np.log2(n)))
    ef = max(1, int(round(k / 2)))
    return rmat_graph(scale, ef, sub, wrange=wrange, n=n, name=f"batch{gi}_rmat_n{n}")


def batched_suite(count: int = 256, seed0: int = 1000, nmin: int = 200,
                  nmax: int = 20000, kmin: float = 4, kmax: float = 64,
                  wrange=(1, 100)) -> list:
    """Many independent graphs of uneven sizes, kinds and densities, weights
    uniform in ``wrange`` (see batched_specs and batched_graph)."""
    specs = batched_specs(count, seed0, nmin, nmax, kmin, kmax)
    return [batched_graph(gi, sp, wrange) for gi, sp in enumerate(specs)]


def poisson_trace(rate: float, count: int, n_graphs: int, seed: int,
                  smin: int = 16, smax: int = 1024):
    """Request arrivals: exponential gaps at ``rate`` per second.

    Returns (arrival_seconds float64[count], graph_index int32[count],
    n_sources int32[count]) with the source count log-uniform integer in
    [smin, smax] and the graph uniform over ``n_graphs``.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    gidx = rng.integers(0, n_graphs, size=count).astype(np.int32)
    ns = np.exp(rng.uniform(np.log(smin), np.log(smax + 1), size=count))
    ns = np.clip(np.floor(ns), smin, smax).astype(np.int32)
    return t, gidx, ns


# ---------------------------------------------------------------- directed graphs
@dataclass
class DiGraph:
    """Directed simple graph: out-arc CSR (row u lists the heads of u's arcs)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray]
    name: str = ""

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def directed_rmat_graph(scale: int, ef: int, seed: int, abcd=(0.57, 0.19, 0.19, 0.05),
                        wrange=None, name: str = "") -> DiGraph:
    """Directed R-MAT: ``ef * 2**scale`` arcs, loops and duplicate arcs dropped, ids permuted."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    u, v = _rmat_pairs(rng, scale, ef * n, abcd)
    keep = u != v
    key = np.unique(u[keep] * np.int64(n) + v[keep])
    perm = rng.permutation(n).astype(np.int64)
    u, v = perm[key // n], perm[key % n]
    order = np.lexsort((v, u))
    u, v = u[order], v[order]
    w = _draw_weights(rng, u.size, wrange)
    counts = np.bincount(u, minlength=n)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return DiGraph(n, row_ptr, v.astype(np.int32), w, name or f"drmat_s{scale}_ef{ef}_s{seed}")
