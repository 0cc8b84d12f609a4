// Host-side work decomposition of libmfbc.
//
// A CSR orientation is cut into pull tasks for one wave each: runs of
// consecutive light rows (bounded total arcs and at most 64 rows, so a run's
// activity fits one 64-bit mask), and fixed-size slices of heavy rows (the
// hubs of power-law graphs), whose partial results are merged in slice order
// by a second kernel.  Balancing the arcs per task keeps one wave from
// walking a 10^5-arc hub row while the rest of the GPU idles.
#include <algorithm>

#include "mfbc_internal.h"

namespace mfbc {

TaskParams default_params(int32_t n, int64_t arcs) {
    // Aim for enough tasks to fill the GPU many times over (256 CUs x 64
    // waves), shrinking runs on small graphs where a long serial run would
    // make one product latency-bound.
    constexpr int64_t kTarget = 16384;
    TaskParams p;
    p.run_verts = (int)std::min<int64_t>(64, std::max<int64_t>(1, (n + kTarget - 1) / kTarget));
    p.run_arcs = (int)std::min<int64_t>(512, std::max<int64_t>(64, (arcs + kTarget - 1) / kTarget));
    return p;
}

int build_plan(int32_t n, const int64_t *rp, const TaskParams &p, std::vector<Task> &tasks,
               std::vector<Hub> &hubs, int32_t &nslots) {
    tasks.clear();
    hubs.clear();
    nslots = 0;
    const int run_verts = std::min(std::max(p.run_verts, 1), 64);
    const int64_t heavy = std::max(p.heavy, 1);
    const int64_t slice = std::max(p.slice, 1);
    const int64_t run_arcs = std::max(p.run_arcs, 1);
    int32_t v = 0;
    while (v < n) {
        const int64_t d = rp[v + 1] - rp[v];
        if (d > heavy) {
            const int32_t np = (int32_t)((d + slice - 1) / slice);
            Hub h{v, nslots, np, 0};
            const int32_t hid = (int32_t)hubs.size();
            hubs.push_back(h);
            for (int32_t k = 0; k < np; k++) {
                Task t{};
                t.v0 = v;
                t.v1 = v + 1;
                t.hub = hid;
                t.part = nslots + k;
                t.e0 = rp[v] + (int64_t)k * slice;
                t.e1 = std::min(rp[v] + (int64_t)(k + 1) * slice, rp[v + 1]);
                tasks.push_back(t);
            }
            nslots += np;
            v++;
            continue;
        }
        const int32_t v0 = v;
        int64_t arcs = 0;
        while (v < n && v - v0 < run_verts) {
            const int64_t dv = rp[v + 1] - rp[v];
            if (dv > heavy) break;
            if (v > v0 && arcs + dv > run_arcs) break;
            arcs += dv;
            v++;
        }
        Task t{};
        t.v0 = v0;
        t.v1 = v;
        t.hub = -1;
        t.part = -1;
        t.e0 = rp[v0];
        t.e1 = rp[v];
        tasks.push_back(t);
    }
    return 0;
}

}  // namespace mfbc
