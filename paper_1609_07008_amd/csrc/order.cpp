// Host-side CSR checks and reorganisation (see order.h).
#include "order.h"

#include <algorithm>

#include "../../include/mfbc.h"

namespace mfbc {

int validate_csr(int32_t n, int64_t n_arcs, const int64_t *rp, const int32_t *col,
                 const int32_t *w, int32_t *maxw, std::string &msg) {
    if (n < 1 || n == INT32_MAX) {
        msg = "n must be in [1, 2^31 - 2]";
        return MFBC_EINVAL;
    }
    if (n_arcs < 0) {
        msg = "n_arcs must be >= 0";
        return MFBC_EINVAL;
    }
    if (!rp) {
        msg = "row_ptr is NULL";
        return MFBC_EINVAL;
    }
    if (n_arcs > 0 && !col) {
        msg = "col_idx is NULL";
        return MFBC_EINVAL;
    }
    if (rp[0] != 0 || rp[n] != n_arcs) {
        msg = "row_ptr[0] must be 0 and row_ptr[n] must equal n_arcs";
        return MFBC_EINVAL;
    }
    int32_t mw = 1;
    for (int32_t v = 0; v < n; v++) {
        if (rp[v + 1] < rp[v] || rp[v + 1] > n_arcs) {
            msg = "row_ptr must be non-decreasing and end at n_arcs";
            return MFBC_EINVAL;
        }
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            const int32_t c = col[e];
            if (c < 0 || c >= n) {
                msg = "column index out of range";
                return MFBC_EINVAL;
            }
            if (c == v) {
                msg = "self-loop at vertex " + std::to_string(v);
                return MFBC_EINVAL;
            }
            if (e > rp[v] && col[e - 1] >= c) {
                msg = "row " + std::to_string(v) + " is not strictly increasing (duplicate arc?)";
                return MFBC_EINVAL;
            }
            if (w) {
                if (w[e] < 1) {
                    msg = "weights must be >= 1";
                    return MFBC_EINVAL;
                }
                mw = std::max(mw, w[e]);
            }
        }
    }
    if ((int64_t)n * (int64_t)mw >= (int64_t)INT32_MAX) {
        msg = "n * max weight does not fit int32 distances";
        return MFBC_EOVERFLOW;
    }
    *maxw = mw;
    return MFBC_OK;
}

bool is_symmetric(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col, const int32_t *w,
                  const std::vector<int64_t> &rpt, const std::vector<int32_t> &colt,
                  const std::vector<int32_t> &wt) {
    if (rpt.size() != (size_t)n + 1 || colt.size() != (size_t)arcs) return false;
    return std::equal(rpt.begin(), rpt.end(), rp) && std::equal(colt.begin(), colt.end(), col) &&
           (!w || std::equal(wt.begin(), wt.end(), w));
}

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
