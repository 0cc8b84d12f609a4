// Test harness for the host-side work decomposition (graph.cpp): reads a
// row-pointer array and the decomposition parameters from argv[1], writes
// the default parameters for (n, arcs), the tasks, the hubs and the slot
// count to argv[2].  Layout of both files: see test_host_plan.py.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "mfbc_internal.h"

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int32_t n = 0, prm[4] = {0, 0, 0, 0};
    if (fread(&n, 4, 1, in) != 1 || fread(prm, 4, 4, in) != 4) return 3;
    std::vector<int64_t> rp((size_t)n + 1);
    if (fread(rp.data(), 8, rp.size(), in) != rp.size()) return 3;
    fclose(in);
    mfbc::TaskParams p;
    p.run_arcs = prm[0];
    p.run_verts = prm[1];
    p.heavy = prm[2];
    p.slice = prm[3];
    std::vector<mfbc::Task> tasks;
    std::vector<mfbc::Hub> hubs;
    int32_t nslots = 0;
    mfbc::build_plan(n, rp.data(), p, tasks, hubs, nslots);
    const mfbc::TaskParams d = mfbc::default_params(n, rp[(size_t)n]);
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    const int32_t head[5] = {d.run_arcs, d.run_verts, (int32_t)tasks.size(), (int32_t)hubs.size(), nslots};
    fwrite(head, 4, 5, out);
    for (const auto &t : tasks) {
        const int32_t a[4] = {t.v0, t.v1, t.hub, t.part};
        const int64_t e[2] = {t.e0, t.e1};
        fwrite(a, 4, 4, out);
        fwrite(e, 8, 2, out);
    }
    for (const auto &h : hubs) {
        const int32_t a[3] = {h.v, h.first, h.nparts};
        fwrite(a, 4, 3, out);
    }
    fclose(out);
    return 0;
}
