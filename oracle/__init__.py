"""CPU oracle for MFBC parity -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (``libmfbc`` and its
Python binding) never imports, links or runs anything here, and nothing here
imports the product path: the only module both sides use is the seeded input
generator ``paper_1609_07008_amd.graphgen``, which holds no arithmetic of the
method.

Contents
  brandes   -- Brandes' algorithm in C (FP64), Section 2.4: tau, sigma, delta,
               lambda, plus shortest-path-DAG heights.
  brute     -- exhaustive enumeration of simple paths / walks on tiny graphs
               (exact rational arithmetic), the pin for everything else.
  frontier  -- the frontier sets MFBF (Algorithm 1) and MFBr (Algorithm 2)
               must produce, from their definitions (Lemma 1: hop-indexed
               least-weight walks; Lemma 2: shortest-path-DAG heights), the
               product counts and relaxations that follow from them, and the
               monoid fixpoints (SSSP / BFS) of Section 3's product.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(brute force, closed forms, invariants, an independent library); none is
"parity unpinned" except sigma values beyond 2**53 on irregular graphs, where
binary64 summation order matters and only a relative bound applies.
"""
from .brandes import brandes, brandes_threads, build_library, library_path  # noqa: F401
from .frontier import (backward_heights, backward_products, forward_frontiers,  # noqa: F401
                       forward_relaxations)
from . import brute  # noqa: F401,E402
