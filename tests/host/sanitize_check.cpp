// Sanitizer harness for the host-side code of libmfbc that runs before any
// device work: the CSR validation (order.cpp: validate_csr, is_symmetric),
// the transpose and descending-degree renumbering (order.cpp) and the work
// decomposition (graph.cpp).  Built with g++ -fsanitize=address,undefined by
// tests/test_host_sanitize.py.  argv[1] holds a sequence of cases, each:
//   int32 n, int64 n_arcs, int32 has_weights, int32 undirected,
//   int64 row_ptr[n+1], int32 col[n_arcs], int32 w[n_arcs] (if has_weights);
// every array is copied into a heap block of exactly its size, so that any
// read past the caller's arrays is reported.  argv[2] receives, per case,
// int32 status (0, or the MFBC_E* code), int32 max weight, int32 symmetric,
// int32 tasks, int32 hubs, int32 slots (the last four 0 unless status is 0).
#include <cstdio>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "mfbc_internal.h"
#include "order.h"

template <typename T>
static bool get(FILE *f, T *p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    FILE *out = fopen(argv[2], "wb");
    if (!in || !out) return 2;
    for (;;) {
        int32_t n = 0, hasw = 0, undirected = 0;
        int64_t arcs = 0;
        if (!get(in, &n, 1)) break;
        if (!get(in, &arcs, 1) || !get(in, &hasw, 1) || !get(in, &undirected, 1)) return 3;
        const size_t nrp = n >= 0 ? (size_t)n + 1 : 0, na = arcs > 0 ? (size_t)arcs : 0;
        std::unique_ptr<int64_t[]> rp(new int64_t[nrp]);
        std::unique_ptr<int32_t[]> col(new int32_t[na]), w(hasw ? new int32_t[na] : nullptr);
        if (!get(in, rp.get(), nrp) || !get(in, col.get(), na)) return 3;
        if (hasw && !get(in, w.get(), na)) return 3;
        int32_t res[6] = {0, 0, 0, 0, 0, 0};
        std::string msg;
        int32_t maxw = 0;
        res[0] = mfbc::validate_csr(n, arcs, rp.get(), na ? col.get() : nullptr, w.get(), &maxw, msg);
        if (res[0] == 0) {
            res[1] = maxw;
            std::vector<int64_t> rpt, rpr, rpo;
            std::vector<int32_t> colt, wt, perm, iperm, colr, wr, colo, wo;
            mfbc::build_transpose(n, arcs, rp.get(), col.get(), w.get(), rpt, colt, wt);
            res[2] = mfbc::is_symmetric(n, arcs, rp.get(), col.get(), w.get(), rpt, colt, wt);
            mfbc::degree_order(n, arcs, rp.get(), col.get(), perm, iperm);
            mfbc::relabel_reverse(n, arcs, rp.get(), col.get(), w.get(), perm, iperm, rpr, colr, wr);
            mfbc::build_transpose(n, arcs, rpr.data(), colr.data(), hasw ? wr.data() : nullptr, rpo,
                                  colo, wo);
            const mfbc::TaskParams plans[3] = {mfbc::default_params(n, arcs), {64, 1, 2, 1},
                                               {700, 3, 40, 7}};
            for (const auto &p : plans) {
                std::vector<mfbc::Task> tasks;
                std::vector<mfbc::Hub> hubs;
                int32_t slots = 0;
                mfbc::build_plan(n, rpr.data(), p, tasks, hubs, slots);
                res[3] += (int32_t)tasks.size();
                res[4] += (int32_t)hubs.size();
                res[5] += slots;
            }
        } else if (msg.empty()) {
            return 4;                 // every rejection carries a message
        }
        fwrite(res, sizeof(res), 1, out);
    }
    fclose(in);
    fclose(out);
    return 0;
}
