"""Exhaustive enumeration on tiny graphs -- test infrastructure only.

The definitions of Section 2.4 evaluated literally, with exact integers and
rationals: every simple path from s is enumerated, tau(s,t) is the least
weight, sigma(s,t) the number of least-weight paths, sigma(s,t,v) the number
of those passing through v as an interior vertex, delta(s,v) =
sum_t sigma(s,t,v)/sigma(s,t) and lambda(v) = sum_s delta(s,v).  Positive
weights make every shortest walk a simple path, so simple paths suffice.

Also: least-weight j-arc *walks* by enumeration (the pin of the forward
frontier closed form) and shortest-path-DAG heights by enumeration of DAG
paths (the pin of the backward frontiers).  Intended for n <= 12.
"""
from __future__ import annotations

from fractions import Fraction


def _adj(g):
    adj = [[] for _ in range(g.n)]
    for x in range(g.n):
        for e in range(int(g.row_ptr[x]), int(g.row_ptr[x + 1])):
            wt = 1 if g.w is None else int(g.w[e])
            adj[x].append((int(g.col[e]), wt))
    return adj


def simple_paths(g, s):
    """Yield (path tuple, weight) for every simple path starting at s (including (s,))."""
    adj = _adj(g)
    stack = [((s,), 0, {s})]
    while stack:
        path, wt, seen = stack.pop()
        yield path, wt
        for y, w in adj[path[-1]]:
            if y not in seen:
                stack.append((path + (y,), wt + w, seen | {y}))


def brute_bc(g, sources):
    """Exact tau, sigma, delta per source and lambda; unreachable tau = None."""
    n = g.n
    lam = [Fraction(0)] * n
    per = []
    for s in sources:
        best = {}
        for path, wt in simple_paths(g, s):
            t = path[-1]
            if t not in best or wt < best[t][0]:
                best[t] = [wt, [path]]
            elif wt == best[t][0]:
                best[t][1].append(path)
        tau = [None] * n
        sig = [0] * n
        through = [[0] * n for _ in range(n)]     # through[t][v]
        for t, (wt, paths) in best.items():
            tau[t] = wt
            sig[t] = len(paths)
            for p in paths:
                for v in p[1:-1]:
                    through[t][v] += 1
        delta = [Fraction(0)] * n
        for v in range(n):
            if v == s:
                continue
            acc = Fraction(0)
            for t in range(n):
                if t != s and t != v and sig[t] > 0 and through[t][v]:
                    acc += Fraction(through[t][v], sig[t])
            delta[v] = acc
            lam[v] += acc
        per.append({"tau": tau, "sigma": sig, "delta": delta})
    return per, lam


def walk_minima(g, s, jmax):
    """l_j(v) and the number of least-weight j-arc walks, j = 0..jmax, by enumeration."""
    adj = _adj(g)
    layers = [{s: [(0, 1)]}]
    ell, cnt = [], []
    frontier = {s: {0: 1}}                   # vertex -> {weight: number of walks}
    for j in range(jmax + 1):
        lj = [None] * g.n
        cj = [0] * g.n
        for v, ws in frontier.items():
            m = min(ws)
            lj[v] = m
            cj[v] = ws[m]
        ell.append(lj)
        cnt.append(cj)
        nxt = {}
        for x, ws in frontier.items():
            for y, w in adj[x]:
                d = nxt.setdefault(y, {})
                for wt, c in ws.items():
                    d[wt + w] = d.get(wt + w, 0) + c
        frontier = nxt
    del layers
    return ell, cnt


def dag_heights(g, s, tau):
    """Longest arc count from v down to a sink of s's shortest-path DAG (None if unreachable)."""
    adj = _adj(g)
    n = g.n
    memo = {}

    def h(v):
        if v in memo:
            return memo[v]
        best = 0
        for y, w in adj[v]:
            if tau[y] is not None and tau[v] + w == tau[y]:
                best = max(best, 1 + h(y))
        memo[v] = best
        return best

    return [None if tau[v] is None else h(v) for v in range(n)]


def simple_path_arcs(g, s):
    """Yield (path tuple, [arc weights in path order]) for every simple path
    starting at s (including (s,) with no arcs)."""
    adj = _adj(g)
    stack = [((s,), (), {s})]
    while stack:
        path, ws, seen = stack.pop()
        yield path, list(ws)
        for y, w in adj[path[-1]]:
            if y not in seen:
                stack.append((path + (y,), ws + (w,), seen | {y}))


def walk_best(g, s, jmax, fold, better, start):
    """best[j][v]: the best, by `better(a, b)` (a strictly better than b), of
    fold(...fold(fold(start, w1), w2)..., wj) over every walk from s to v with
    exactly j arcs, j = 0..jmax (None where no such walk), by enumerating the
    walks one by one (no recurrence over j)."""
    adj = _adj(g)
    best = [[None] * g.n for _ in range(jmax + 1)]
    stack = [(s, start, 0)]
    while stack:
        v, val, j = stack.pop()
        if best[j][v] is None or better(val, best[j][v]):
            best[j][v] = val
        if j < jmax:
            for y, w in adj[v]:
                stack.append((y, fold(val, w), j + 1))
    return best
