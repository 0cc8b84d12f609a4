// Host-side CSR reorganisation of libmfbc (no device code): the transpose
// of a CSR and the descending-degree vertex numbering the device copy of a
// graph uses.  Plain C++, so the tests can build and check it on the CPU.
#pragma once

#include <stdint.h>

#include <vector>

namespace mfbc {

// Transpose of a CSR (row c lists u for every arc u -> c, ascending, with
// the weights when w is not NULL).
void build_transpose(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                     const int32_t *w, std::vector<int64_t> &rpt, std::vector<int32_t> &colt,
                     std::vector<int32_t> &wt);

// Descending-degree vertex order (in- plus out-degree, ties by id):
// perm[v] = position of caller vertex v, iperm = its inverse.
void degree_order(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                  std::vector<int32_t> &perm, std::vector<int32_t> &iperm);

// Reverse graph in the new numbering: row perm[x] lists perm[u] for every
// arc u -> x, ascending, with the weights when w is not NULL.
void relabel_reverse(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                     const int32_t *w, const std::vector<int32_t> &perm,
                     const std::vector<int32_t> &iperm, std::vector<int64_t> &rpr,
                     std::vector<int32_t> &colr, std::vector<int32_t> &wr);

}  // namespace mfbc
