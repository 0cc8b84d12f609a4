"""Expected per-product values of the forward loop, from the oracle's
frontier definitions (Lemma 1), for comparisons with traced GPU runs."""
import numpy as np

from oracle import frontier


def expected_forward(g, sources, arcs=None):
    """Frontier sets and relaxations the forward loop of one batch must give.

    Returns (products, member, nnz, relax): products = the first product whose
    frontier is empty in every column; member(j) -> bool[nb][n], F_j per
    column (j = 1..products); nnz[j-1] = |F_j|; relax[j-1] = relaxations of
    product j (arcs leaving F_{j-1})."""
    arcs = arcs or frontier.InArcs(g)
    per = [frontier.forward_frontiers(g, int(s), arcs=arcs) for s in sources]
    products = max(len(x) for x in per)
    empty = np.zeros(g.n, dtype=bool)

    def member(j):
        return np.stack([x[j - 1] if j <= len(x) else empty for x in per])

    nnz = [int(sum(int(x[j - 1].sum()) for x in per if j <= len(x))) for j in range(1, products + 1)]
    rel = [frontier.forward_relaxations(g, int(s), x, arcs=arcs) for s, x in zip(sources, per)]
    relax = [int(sum(r[j - 1] for r in rel if j <= len(r))) for j in range(1, products + 1)]
    return products, member, nnz, relax
