// Test harness for the host-side CSR reorganisation (order.cpp): reads a CSR
// from argv[1], writes the descending-degree numbering and the relabelled
// reverse CSR (and, for a directed graph, its transpose: the relabelled
// out-arc CSR) to argv[2].  Layout of both files: see test_host_order.py.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "order.h"

template <typename T>
static bool get(FILE *f, T *p, size_t n) { return fread(p, sizeof(T), n, f) == n; }
template <typename T>
static void put(FILE *f, const T *p, size_t n) { fwrite(p, sizeof(T), n, f); }

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int32_t n = 0, weighted = 0, directed = 0;
    int64_t arcs = 0;
    if (!get(in, &n, 1) || !get(in, &arcs, 1) || !get(in, &weighted, 1) || !get(in, &directed, 1))
        return 3;
    std::vector<int64_t> rp((size_t)n + 1);
    std::vector<int32_t> col((size_t)arcs), w(weighted ? (size_t)arcs : 0);
    if (!get(in, rp.data(), rp.size()) || !get(in, col.data(), col.size())) return 3;
    if (weighted && !get(in, w.data(), w.size())) return 3;
    fclose(in);
    const int32_t *wp = weighted ? w.data() : nullptr;
    std::vector<int32_t> perm, iperm, colr, wr, colo, wo;
    std::vector<int64_t> rpr, rpo;
    mfbc::degree_order(n, arcs, rp.data(), col.data(), perm, iperm);
    mfbc::relabel_reverse(n, arcs, rp.data(), col.data(), wp, perm, iperm, rpr, colr, wr);
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    put(out, perm.data(), perm.size());
    put(out, rpr.data(), rpr.size());
    put(out, colr.data(), colr.size());
    if (weighted) put(out, wr.data(), wr.size());
    if (directed) {
        mfbc::build_transpose(n, arcs, rpr.data(), colr.data(), weighted ? wr.data() : nullptr, rpo,
                              colo, wo);
        put(out, rpo.data(), rpo.size());
        put(out, colo.data(), colo.size());
        if (weighted) put(out, wo.data(), wo.size());
    }
    fclose(out);
    return 0;
}
