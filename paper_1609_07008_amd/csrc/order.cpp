// Host-side CSR reorganisation (see order.h).
#include "order.h"

#include <algorithm>

namespace mfbc {

// Also the symmetry check of an undirected CSR (the transpose must equal it).
void build_transpose(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                     const int32_t *w, std::vector<int64_t> &rpt, std::vector<int32_t> &colt,
                     std::vector<int32_t> &wt) {
    rpt.assign((size_t)n + 1, 0);
    for (int64_t e = 0; e < arcs; e++) rpt[(size_t)col[e] + 1]++;
    for (int32_t v = 0; v < n; v++) rpt[(size_t)v + 1] += rpt[(size_t)v];
    colt.assign((size_t)arcs, 0);
    if (w) wt.assign((size_t)arcs, 0);
    std::vector<int64_t> pos(rpt.begin(), rpt.end() - 1);
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            const int64_t p = pos[(size_t)col[e]]++;
            colt[(size_t)p] = u;
            if (w) wt[(size_t)p] = w[e];
        }
}

// Descending-degree vertex order (in- plus out-degree, ties by id):
// perm[v] = position of caller vertex v, iperm = its inverse.
void degree_order(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                  std::vector<int32_t> &perm, std::vector<int32_t> &iperm) {
    std::vector<int64_t> key((size_t)n, 0);
    for (int32_t v = 0; v < n; v++) key[(size_t)v] += rp[v + 1] - rp[v];
    for (int64_t e = 0; e < arcs; e++) key[(size_t)col[e]]++;
    iperm.resize((size_t)n);
    for (int32_t v = 0; v < n; v++) iperm[(size_t)v] = v;
    std::stable_sort(iperm.begin(), iperm.end(),
                     [&](int32_t a, int32_t b) { return key[(size_t)a] > key[(size_t)b]; });
    perm.resize((size_t)n);
    for (int32_t r = 0; r < n; r++) perm[(size_t)iperm[(size_t)r]] = r;
}

// Reverse graph in the new numbering: row perm[x] lists perm[u] for every
// arc u -> x, ascending (rows are visited in new-id order), with the weights.
void relabel_reverse(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col,
                     const int32_t *w, const std::vector<int32_t> &perm,
                     const std::vector<int32_t> &iperm, std::vector<int64_t> &rpr,
                     std::vector<int32_t> &colr, std::vector<int32_t> &wr) {
    rpr.assign((size_t)n + 1, 0);
    for (int64_t e = 0; e < arcs; e++) rpr[(size_t)perm[(size_t)col[e]] + 1]++;
    for (int32_t v = 0; v < n; v++) rpr[(size_t)v + 1] += rpr[(size_t)v];
    colr.assign((size_t)arcs, 0);
    if (w) wr.assign((size_t)arcs, 0);
    std::vector<int64_t> pos(rpr.begin(), rpr.end() - 1);
    for (int32_t r = 0; r < n; r++) {
        const int32_t u = iperm[(size_t)r];
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            const int64_t p = pos[(size_t)perm[(size_t)col[e]]]++;
            colr[(size_t)p] = r;
            if (w) wr[(size_t)p] = w[e];
        }
    }
}

}  // namespace mfbc
