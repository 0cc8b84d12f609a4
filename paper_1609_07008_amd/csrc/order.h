// Host-side CSR checks and reorganisation of libmfbc (no device code): the
// validation of a caller's CSR, the transpose of a CSR and the
// descending-degree vertex numbering the device copy of a graph uses.  Plain
// C++, so the tests can build and check it on the CPU (also under the
// address and undefined-behaviour sanitizers).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace mfbc {

// Validation of a caller's CSR before any device work (the rules of
// mfbc_load_graph): n in [1, 2^31 - 2], n_arcs >= 0, row_ptr[0] = 0,
// non-decreasing, row_ptr[n] = n_arcs, columns in [0, n), strictly increasing
// per row (no duplicate arcs), no self-loops, weights >= 1 (NULL: all 1), and
// n * max weight below 2^31 - 1 (int32 distances).  Returns 0 and the
// largest weight, or MFBC_EINVAL / MFBC_EOVERFLOW with a message.  Reads no
// entry of a row before its row pointers are known to lie in [0, n_arcs].
int validate_csr(int32_t n, int64_t n_arcs, const int64_t *rp, const int32_t *col,
                 const int32_t *w, int32_t *maxw, std::string &msg);

// Whether an undirected CSR is symmetric with equal weights on both arcs,
// given its transpose (rpt, colt, wt from build_transpose).
bool is_symmetric(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col, const int32_t *w,
                  const std::vector<int64_t> &rpt, const std::vector<int32_t> &colt,
                  const std::vector<int32_t> &wt);

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
