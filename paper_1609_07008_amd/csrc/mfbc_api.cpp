// C ABI of libmfbc (declared in include/mfbc.h): validation, device memory,
// and the host loops of Algorithms 1-3 around the HIP kernels.
//
// Per batch (Algorithm 3): initialise T and the first frontier (the sources
// themselves), then repeat the forward product until a product yields an
// empty frontier (Algorithm 1's loop condition, over all columns of the
// batch); then the counting product and the backward products until the
// backward frontier is empty (Algorithm 2); lambda parts are accumulated by
// the kernels as entries complete.  The size of each new frontier is read
// back after every product (a 256-byte copy and a stream synchronisation);
// that is the only host round trip of the loop.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "mfbc_internal.h"
#include "order.h"

using namespace mfbc;

// Scratch of mfbc_bc_noalloc: one file-scope device array per GPU (the code
// object's copy on each device), holding the workspace of one call.  Calls on
// one device share it; each call initialises what it reads.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace

int mfbc::set_error(int code, const std::string &msg) { return fail(code, msg); }

namespace {

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(MFBC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(MFBC_ENOMEM, std::string("device allocation of ") +
                                     std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return MFBC_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// Every array of the per-batch workspace for `ncg` column groups, in a fixed
// order: f(pointer, element count).  Used both to allocate the arrays and to
// carve them out of one block of memory.
// (g == nullptr: every count is 0, for walks that need only the pointers.)
template <typename F>
void ws_arrays(const mfbc_graph *g, Workspace &ws, int ncg, F &&f) {
    const size_t n = g ? (size_t)g->n : 0;
    const size_t tile = n * kWave * (size_t)ncg;
    const size_t nwords = (n + 31) / 32;
    const size_t slots =
        g ? (size_t)std::max(g->plan_in.nslots, g->plan_out.nslots) * kWave * (size_t)ncg : 0;
    f(ws.tdist, tile);
    f(ws.tsig, tile);
    for (int b = 0; b < 2; b++) {
        f(ws.fdist[b], tile);
        f(ws.fsig[b], tile);
        f(ws.fbits[b], n * ncg);
        f(ws.abits[b], nwords * ncg);
    }
    f(ws.pd, slots);
    f(ws.pm, slots);
    f(ws.counters, (size_t)kCounterRing * 4 * kCounterSlots);
    f(ws.flags, (size_t)4);
    f(ws.lam, n * ncg);
    f(ws.dag, (size_t)std::max<int64_t>(g ? g->arcs : 0, 1) * ncg);
    f(ws.src, (size_t)ncg * kWave);
    f(ws.tau2, ncg >= 2 ? tile / 2 : (size_t)1);   // the paired counting product's 16-bit tau
}

// Column groups the workspace holds for a batch of `ncg` groups: batches of
// two or more run the forward product on pairs, so their count is rounded up
// to whole pairs; a single group runs alone.
int ws_groups(int ncg) { return ncg <= 1 ? 1 : (ncg + 1) & ~1; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bytes of the workspace of `ncg` groups when carved from one block.
size_t ws_bytes(const mfbc_graph *g, int ncg) {
    Workspace tmp;
    size_t off = 0;
    ws_arrays(g, tmp, ws_groups(ncg), [&](auto *&p, size_t count) {
        (void)p;
        off = align256(off + std::max<size_t>(count, 1) * sizeof(*p));
    });
    return off;
}

void free_workspace(Workspace &ws) {
    if (!ws.external) ws_arrays(nullptr, ws, 0, [](auto *&p, size_t) { dfree(p); });
    dfree(ws.trace_relax);
    ws = Workspace{};
}

void free_plan(Plan &p) {
    dfree(p.tasks);
    dfree(p.hubs);
    p.ntasks = p.nhubs = p.nslots = 0;
}

int upload_plan(int32_t n, const int64_t *h_rp, const TaskParams &prm, Plan &plan) {
    std::vector<Task> tasks;
    std::vector<Hub> hubs;
    int32_t nslots = 0;
    build_plan(n, h_rp, prm, tasks, hubs, nslots);
    free_plan(plan);
    int rc;
    if ((rc = dalloc(&plan.tasks, tasks.size()))) return rc;
    if ((rc = dalloc(&plan.hubs, hubs.size()))) return rc;
    if (!tasks.empty())
        HIP_TRY(hipMemcpy(plan.tasks, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice));
    if (!hubs.empty())
        HIP_TRY(hipMemcpy(plan.hubs, hubs.data(), hubs.size() * sizeof(Hub), hipMemcpyHostToDevice));
    plan.ntasks = (int32_t)tasks.size();
    plan.nhubs = (int32_t)hubs.size();
    plan.nslots = nslots;
    return MFBC_OK;
}

// Grow the workspace to hold a batch of `ncg` column groups.
int ensure_workspace(mfbc_graph *g, int ncg) {
    Workspace &ws = g->ws;
    ncg = ws_groups(ncg);
    if (ws.ncg >= ncg && !ws.external) return MFBC_OK;
    free_workspace(ws);
    int rc = MFBC_OK;
    ws_arrays(g, ws, ncg, [&](auto *&p, size_t count) {
        if (!rc) rc = dalloc(&p, count);
    });
    if (rc) {
        free_workspace(ws);
        return rc;
    }
    ws.ncg = ncg;
    return MFBC_OK;
}

struct Counts {
    int64_t produced = 0, outputs = 0, active_vertices = 0, active_arcs = 0;
};

// Wait for the stream and copy the whole counter ring to the host.
int read_ring(mfbc_graph *g, hipStream_t s) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(g->h_ctr, g->ws.counters,
                           sizeof(unsigned long long) * kCounterRing * 4 * kCounterSlots,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

// Counters of product `idx` from the host copy of the ring (see flush_counts).
Counts ring_counts(const mfbc_graph *g, int idx) {
    const size_t off = (size_t)(idx % kCounterRing) * 4 * kCounterSlots;
    int64_t t[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; k++)
        for (int i = 0; i < kCounterSlots; i++) t[k] += (int64_t)g->h_ctr[off + k * kCounterSlots + i];
    Counts c;
    c.produced = t[0];
    c.outputs = t[1];
    c.active_vertices = t[2];
    c.active_arcs = t[3];
    return c;
}

// Kernel times of the product launched in window position `i` (events
// recorded by the launchers).
// Kernel times of window position i: product kernel into *a, its merge into
// *b.  `fwd`: a forward or fixpoint product (timed in both timing modes).
void add_times(mfbc_graph *g, int i, double *a, double *b, bool fwd) {
    if (!g->timing || (g->timing == 2 && !fwd)) return;
    hipEvent_t *e = g->ev + 3 * i;
    float t0 = 0.f, t1 = 0.f;
    if (hipEventElapsedTime(&t0, e[0], e[1]) == hipSuccess) *a += t0;
    if (g->timing == 1 && hipEventElapsedTime(&t1, e[1], e[2]) == hipSuccess) *b += t1;
}

// Events for the launch at window position i (null: not timed).  Timing
// mode 2 records only the two around a forward or fixpoint product kernel:
// every event costs the stream a few microseconds, which small graphs'
// steps feel.
hipEvent_t *window_events(mfbc_graph *g, int i, bool fwd) {
    if (g->timing == 1) return g->ev + 3 * i;
    if (g->timing == 2 && fwd) return g->ev_pull + 3 * i;
    return nullptr;
}

int check_sources(mfbc_graph *g, const int32_t *d_sources, int64_t count, hipStream_t s) {
    if (count == 0) return MFBC_OK;
    if (!d_sources) return fail(MFBC_EINVAL, "sources pointer is NULL");
    std::vector<int32_t> h((size_t)count);
    HIP_TRY(hipMemcpyAsync(h.data(), d_sources, (size_t)count * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < count; i++)
        if (h[(size_t)i] < 0 || h[(size_t)i] >= g->n)
            return fail(MFBC_EINVAL, "source " + std::to_string(h[(size_t)i]) + " at position " +
                                         std::to_string(i) + " is outside [0, n)");
    return MFBC_OK;
}

// Algorithm 1 on the batch whose sources are already in ws.src.
//
// Products are enqueued kWindow at a time and their counters read back
// once per window: a product whose predecessor produced nothing skips
// itself on the device, so the products past the end of the loop in the
// last window cost a launch each and change nothing.  The loop ends at the
// first product that produced no frontier entry (Algorithm 1's condition
// over every column of the batch).
// Trace (d_rows non-null or h_relax non-null): frontier membership of F_j
// after every product j <= max_products, as vertex bitmaps per column
// (d_rows + (j-1) * nb * words), and the relaxations of every product.
int run_forward(mfbc_graph *g, int ncg, int nb, bool trace, uint64_t *d_rows, int64_t *h_nnz,
                int64_t *h_relax, int max_products, int32_t *products, hipStream_t s) {
    launch_fwd_init(g, ncg, nb, s);
    if (trace) launch_trace_fwd(g, ncg, nb, 0, nullptr, s);
    const double arc_bytes = g->weighted ? 8.0 : 4.0;
    const size_t words = ((size_t)g->n + 63) / 64;
    mfbc_stats &st = g->stats;
    int64_t prev = nb;           // the first frontier: one entry per source column
    int j = 0, last = 0;
    while (!last) {
        if (j > g->n + 1) return fail(MFBC_EDEVICE, "forward products did not converge");
        for (int i = 0; i < kWindow; i++) {
            const int jj = j + 1 + i;
            launch_fwd_product(g, ncg, jj, s, window_events(g, i, true));
            if (trace)
                launch_trace_fwd(g, ncg, nb, jj,
                                 d_rows && jj <= max_products ? d_rows + (size_t)(jj - 1) * nb * words
                                                              : nullptr,
                                 s);
        }
        int rc = read_ring(g, s);
        if (rc) return rc;
        for (int i = 0; i < kWindow; i++) {
            const int jj = j + 1 + i;
            st.fwd_pull_launches++;
            add_times(g, i, &st.fwd_pull_ms, &st.fwd_merge_ms, true);
            if (last) continue;          // skipped on the device
            const Counts c = ring_counts(g, jj);
            if (h_nnz && jj <= max_products) h_nnz[jj - 1] = c.produced;
            st.fwd_entries += c.produced;
            st.fwd_outputs += c.outputs;
            st.fwd_active_vertices += c.active_vertices;
            st.fwd_active_arcs += c.active_arcs;
            st.fwd_alg_bytes += 8.0 * c.active_vertices + arc_bytes * c.active_arcs +
                                12.0 * (double)(prev + c.outputs + c.produced);
            prev = c.produced;
            if (c.produced == 0) last = jj;
        }
        j += kWindow;
    }
    g->stats.fwd_products += last;
    if (products) *products = last;
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, g->ws.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (trace && h_relax) {
        const int k = std::min(last, max_products);
        std::vector<unsigned long long> r((size_t)k + 1, 0ull);
        HIP_TRY(hipMemcpyAsync(r.data(), g->ws.trace_relax, sizeof(unsigned long long) * ((size_t)k + 1),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < k; i++) h_relax[i] = (int64_t)r[(size_t)i];
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (flag) return fail(MFBC_EOVERFLOW, "a shortest-path count overflowed binary64");
    return MFBC_OK;
}

// Algorithm 2 on the batch whose T is in the workspace: the counting
// product (window position 0 of the first window), then backward products
// in windows as in run_forward, until one produces no frontier entry.
int run_backward(mfbc_graph *g, int ncg, int nb, int32_t *products, hipStream_t s) {
    const double arc_bytes = g->weighted ? 8.0 : 4.0;
    mfbc_stats &st = g->stats;
    int64_t prev = 0;
    int k = 0, last = -1;
    while (last < 0) {
        if (k > g->n + 1) return fail(MFBC_EDEVICE, "backward products did not converge");
        for (int i = 0; i < kWindow; i++) {
            const int kk = k + i;
            if (kk == 0) {
                const hipError_t e = launch_bwd_count(g, ncg, s, window_events(g, i, false));
                if (e != hipSuccess)
                    return fail(MFBC_EDEVICE, std::string("counting product: ") + hipGetErrorString(e));
            } else {
                launch_bwd_product(g, ncg, kk, s, window_events(g, i, false));
            }
        }
        int rc = read_ring(g, s);
        if (rc) return rc;
        for (int i = 0; i < kWindow; i++) {
            const int kk = k + i;
            if (kk == 0) {
                const Counts c = ring_counts(g, 0);
                st.bwd_entries += c.produced;
                st.count_launches++;
                // adjacency, tau of every (column, vertex) read once, the
                // stored DAG (one 8-byte lane mask per arc and column group)
                // written, the backward state of every (column, vertex)
                // initialised (counter 4 B, zeta 8 B, frontier index 4 B
                // when traced), and each leaf's sigma read and 1/sigma written
                const double state = g->trace_step ? 16.0 : 12.0;
                st.count_alg_bytes += arc_bytes * (double)g->arcs + 8.0 * g->n +
                                      (8.0 + state) * (double)g->n * nb +
                                      8.0 * (double)g->arcs * ncg + 16.0 * (double)c.produced;
                if (g->timing == 1) {
                    float t = 0.f;
                    if (hipEventElapsedTime(&t, g->ev[0], g->ev[2]) == hipSuccess) st.count_ms += t;
                }
                prev = c.produced;
                if (c.produced == 0) last = 0;
                continue;
            }
            st.bwd_pull_launches++;
            add_times(g, i, &st.bwd_pull_ms, &st.bwd_merge_ms, false);
            if (last >= 0) continue;      // skipped on the device
            const Counts c = ring_counts(g, kk);
            st.bwd_entries += c.produced;
            st.bwd_outputs += c.outputs;
            st.bwd_active_vertices += c.active_vertices;
            st.bwd_active_arcs += c.active_arcs;
            // + the DAG lane mask of every arc with an active head (8 B)
            st.bwd_alg_bytes += 8.0 * c.active_vertices + (arc_bytes + 8.0) * c.active_arcs +
                                12.0 * (double)prev + 24.0 * (double)c.outputs;
            prev = c.produced;
            if (c.produced == 0) last = kk;
        }
        k += kWindow;
    }
    st.bwd_products += last + 1;
    if (products) *products = last + 1;
    return MFBC_OK;
}

int forward_impl(mfbc_graph *g, const int32_t *d_sources, int32_t nb, int32_t *d_dist,
                 double *d_sigma, bool trace, uint64_t *d_rows, int64_t *h_nnz, int64_t *h_relax,
                 int32_t max_products, int32_t *h_products, void *stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (nb < 1) return fail(MFBC_EINVAL, "nb must be >= 1");
    if (!d_dist || !d_sigma) return fail(MFBC_EINVAL, "output pointer is NULL");
    if (trace && max_products < 0) return fail(MFBC_EINVAL, "max_products must be >= 0");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    int rc = check_sources(g, d_sources, nb, s);
    if (rc) return rc;
    const int ncg = (nb + kWave - 1) / kWave;
    if ((rc = ensure_workspace(g, ncg))) return rc;
    if (trace) {
        // relaxations of products 1 .. n + 1 + kWindow (every product a loop can launch)
        const int need = g->n + 2 + kWindow;
        if (g->ws.trace_len < need) {
            dfree(g->ws.trace_relax);
            g->ws.trace_len = 0;
            if ((rc = dalloc(&g->ws.trace_relax, (size_t)need))) return rc;
            g->ws.trace_len = need;
        }
        HIP_TRY(hipMemsetAsync(g->ws.trace_relax, 0, sizeof(unsigned long long) * (size_t)need, s));
        if (d_rows && max_products > 0)
            HIP_TRY(hipMemsetAsync(d_rows, 0,
                                   sizeof(uint64_t) * (size_t)max_products * nb * (((size_t)g->n + 63) / 64),
                                   s));
    }
    g->stats = mfbc_stats{};
    launch_set_sources(g, ncg, nb, d_sources, s);
    if ((rc = run_forward(g, ncg, nb, trace, d_rows, h_nnz, h_relax, max_products, h_products, s)))
        return rc;
    g->stats.batches = 1;
    launch_export_forward(g, ncg, nb, d_dist, d_sigma, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

int backward_impl(mfbc_graph *g, const int32_t *d_sources, int32_t nb, const int32_t *d_dist,
                  const double *d_sigma, double *d_delta, int32_t *d_step, int32_t *h_products,
                  void *stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (nb < 1) return fail(MFBC_EINVAL, "nb must be >= 1");
    if (!d_dist || !d_sigma || !d_delta) return fail(MFBC_EINVAL, "array pointer is NULL");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)stream;
    int rc = check_sources(g, d_sources, nb, s);
    if (rc) return rc;
    const int ncg = (nb + kWave - 1) / kWave;
    if ((rc = ensure_workspace(g, ncg))) return rc;
    g->stats = mfbc_stats{};
    launch_set_sources(g, ncg, nb, d_sources, s);
    launch_import_forward(g, ncg, nb, d_dist, d_sigma, s);
    g->trace_step = d_step != nullptr;
    rc = run_backward(g, ncg, nb, h_products, s);
    g->trace_step = false;
    if (rc) return rc;
    g->stats.batches = 1;
    launch_export_backward(g, ncg, nb, d_delta, d_step, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

int bits_for(int64_t x) {
    int b = 0;
    while (x > 0) {
        b++;
        x >>= 1;
    }
    return b;
}

// Device copy of one CSR orientation; weighted rows also get the packed
// (column | weight << cb) words when both fit 32 bits, halving arc traffic.
int upload_csr(int32_t n, int64_t arcs, const int64_t *rp, const int32_t *col, const int32_t *w,
               int32_t maxw, Csr &c) {
    int rc;
    if ((rc = dalloc(&c.rp, (size_t)n + 1)) || (rc = dalloc(&c.col, (size_t)arcs))) return rc;
    HIP_TRY(hipMemcpy(c.rp, rp, ((size_t)n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    if (arcs) HIP_TRY(hipMemcpy(c.col, col, (size_t)arcs * sizeof(int32_t), hipMemcpyHostToDevice));
    if (w) {
        if ((rc = dalloc(&c.w, (size_t)arcs))) return rc;
        if (arcs) HIP_TRY(hipMemcpy(c.w, w, (size_t)arcs * sizeof(int32_t), hipMemcpyHostToDevice));
        const int cb = std::max(1, bits_for((int64_t)n - 1));
        if (cb + bits_for(maxw) <= 32) {
            std::vector<uint32_t> pk((size_t)arcs);
            for (int64_t e = 0; e < arcs; e++)
                pk[(size_t)e] = (uint32_t)col[e] | ((uint32_t)w[e] << cb);
            if ((rc = dalloc(&c.pk, (size_t)arcs))) return rc;
            if (arcs)
                HIP_TRY(hipMemcpy(c.pk, pk.data(), (size_t)arcs * sizeof(uint32_t),
                                  hipMemcpyHostToDevice));
            c.cb = cb;
        }
    }
    return MFBC_OK;
}

// Release a lane view: its workspace, counters and events (the device graph
// it shares stays with its owner).
void free_shadow(mfbc_graph *sh) {
    for (auto &e : sh->ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    free_workspace(sh->ws);
    if (sh->h_ctr) (void)hipHostFree(sh->h_ctr);
    delete sh;
}

void free_graph_memory(mfbc_graph *g) {
    for (int i = 0; i < kMaxLanes; i++) {
        if (g->shadow[i]) free_shadow(g->shadow[i]);
        g->shadow[i] = nullptr;
        if (g->lane_stream[i]) (void)hipStreamDestroy(g->lane_stream[i]);
        g->lane_stream[i] = nullptr;
    }
    if (g->lane_start) (void)hipEventDestroy(g->lane_start);
    g->lane_start = nullptr;
    for (auto &e : g->ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    g->timing = false;
    free_workspace(g->ws);
    free_plan(g->plan_in);
    free_plan(g->plan_out);
    const bool alias = g->in.rp == g->out.rp;
    dfree(g->out.rp);
    dfree(g->out.col);
    dfree(g->out.w);
    dfree(g->out.pk);
    if (!alias) {
        dfree(g->in.rp);
        dfree(g->in.col);
        dfree(g->in.w);
        dfree(g->in.pk);
    }
    g->in = Csr{};
    dfree(g->perm);
    g->h_perm.clear();
    if (g->h_ctr) (void)hipHostFree(g->h_ctr);
    g->h_ctr = nullptr;
}

// Column groups of the workspace for MFBC over n_sources in batches of `batch`.
int bc_groups(int64_t n_sources, int32_t batch) {
    const int64_t width = std::max<int64_t>(1, std::min<int64_t>(batch, n_sources));
    return (int)((width + kWave - 1) / kWave);
}

// Algorithm 3 over the listed sources with the workspace already in place.
int bc_batches(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources, int32_t batch, int ncg,
               double *d_bc, hipStream_t s) {
    g->stats = mfbc_stats{};
    launch_lambda_zero(g, ncg, s);
    int rc;
    for (int64_t b0 = 0; b0 < n_sources; b0 += batch) {
        const int nb = (int)std::min<int64_t>(batch, n_sources - b0);
        const int bcg = (nb + kWave - 1) / kWave;
        launch_set_sources(g, bcg, nb, d_sources + b0, s);
        if ((rc = run_forward(g, bcg, nb, false, nullptr, nullptr, nullptr, 0, nullptr, s)))
            return rc;
        if ((rc = run_backward(g, bcg, nb, nullptr, s))) return rc;
        g->stats.batches++;
    }
    launch_lambda_reduce(g, ncg, d_bc, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

// Lanes of one mfbc_bc call: independent batches run at once on separate
// streams (each batch's products depend only on its own state), which hides
// the launch and read-back latency of small graphs' products and lets the
// sparse products of one batch share the device with another batch's.
int lanes_for(const mfbc_graph *g, int64_t n_batches, int ncg) {
    int S = g->lanes;
    // by default only where a product is too small to fill the device
    if (S <= 0) S = (double)g->arcs * (double)ncg <= (double)(1 << 24) ? kMaxLanes : 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)S, (int64_t)kMaxLanes, n_batches}));
}

// Lane i of g (i = 0: g itself), created on first use; a view is refreshed
// from g on every call (the plan may have changed).
int lane_graph(mfbc_graph *g, int i, mfbc_graph **out) {
    if (i == 0) {
        *out = g;
        return MFBC_OK;
    }
    mfbc_graph *&sh = g->shadow[i];
    if (!sh) {
        sh = new (std::nothrow) mfbc_graph();
        if (!sh) return fail(MFBC_ENOMEM, "host allocation failed");
        sh->is_shadow = true;
        if (hipHostMalloc((void **)&sh->h_ctr,
                          sizeof(unsigned long long) * kCounterRing * 4 * kCounterSlots) != hipSuccess) {
            sh->h_ctr = nullptr;
            delete sh;
            sh = nullptr;
            return fail(MFBC_ENOMEM, "pinned host allocation failed");
        }
    }
    if (!g->lane_stream[i]) HIP_TRY(hipStreamCreateWithFlags(&g->lane_stream[i], hipStreamNonBlocking));
    sh->device = g->device;
    sh->n = g->n;
    sh->arcs = g->arcs;
    sh->maxw = g->maxw;
    sh->weighted = g->weighted;
    sh->directed = g->directed;
    sh->out = g->out;
    sh->in = g->in;
    sh->plan_out = g->plan_out;
    sh->plan_in = g->plan_in;
    sh->mb = g->mb;
    sh->params = g->params;
    sh->perm = g->perm;
    sh->timing = g->timing;
    if (g->timing && !sh->ev[0]) {
        for (auto &e : sh->ev) HIP_TRY(hipEventCreate(&e));
        for (int i = 0; i < 3 * kWindow; i++) sh->ev_pull[i] = i % 3 == 2 ? nullptr : sh->ev[i];
    }
    *out = sh;
    return MFBC_OK;
}

static_assert(sizeof(mfbc_stats) == 14 * sizeof(int64_t) + 9 * sizeof(double),
              "add_stats walks 14 counters and 9 times / byte counts");

void add_stats(mfbc_stats &a, const mfbc_stats &b) {
    int64_t *ai = &a.fwd_products;
    const int64_t *bi = &b.fwd_products;
    for (int k = 0; k < 14; k++) ai[k] += bi[k];
    double *ad = &a.fwd_pull_ms;
    const double *bd = &b.fwd_pull_ms;
    for (int k = 0; k < 9; k++) ad[k] += bd[k];
}

// Algorithm 3 with batch b on lane b % S: lane 0 on the caller's stream, the
// others on their own streams after the caller's prior work; each lane's
// host loop runs on its own thread; lambda = the lanes' parts, summed in lane
// order (so a call is deterministic for a given lane count).
int bc_lanes(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources, int32_t batch, int ncg,
             int S, double *d_bc, hipStream_t s) {
    mfbc_graph *lg[kMaxLanes] = {};
    hipStream_t ls[kMaxLanes] = {};
    int rc;
    for (int i = 0; i < S; i++) {
        if ((rc = lane_graph(g, i, &lg[i]))) return rc;
        if ((rc = ensure_workspace(lg[i], ncg))) return rc;
        ls[i] = i == 0 ? s : g->lane_stream[i];
    }
    if (!g->lane_start) HIP_TRY(hipEventCreateWithFlags(&g->lane_start, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(g->lane_start, s));
    for (int i = 1; i < S; i++) HIP_TRY(hipStreamWaitEvent(ls[i], g->lane_start, 0));
    const int64_t nbat = (n_sources + batch - 1) / batch;
    int rcs[kMaxLanes] = {};
    std::string msgs[kMaxLanes];
    auto lane = [&](int i) {
        mfbc_graph *x = lg[i];
        int r = MFBC_OK;
        if (hipSetDevice(g->device) != hipSuccess) r = fail(MFBC_EDEVICE, "hipSetDevice failed");
        x->stats = mfbc_stats{};
        if (!r) launch_lambda_zero(x, ncg, ls[i]);
        for (int64_t b = i; !r && b < nbat; b += S) {
            const int64_t b0 = b * batch;
            const int nb = (int)std::min<int64_t>(batch, n_sources - b0);
            const int bcg = (nb + kWave - 1) / kWave;
            launch_set_sources(x, bcg, nb, d_sources + b0, ls[i]);
            if (!r) r = run_forward(x, bcg, nb, false, nullptr, nullptr, nullptr, 0, nullptr, ls[i]);
            if (!r) r = run_backward(x, bcg, nb, nullptr, ls[i]);
            x->stats.batches++;
        }
        if (!r && hipStreamSynchronize(ls[i]) != hipSuccess) r = fail(MFBC_EDEVICE, "lane stream failed");
        rcs[i] = r;
        if (r) msgs[i] = mfbc_last_error();
    };
    std::vector<std::thread> th;
    for (int i = 1; i < S; i++) th.emplace_back(lane, i);
    lane(0);
    for (auto &t : th) t.join();
    for (int i = 0; i < S; i++)
        if (rcs[i]) return fail(rcs[i], msgs[i]);
    launch_lambda_reduce_lanes(lg, S, ncg, d_bc, s);
    mfbc_stats tot{};
    for (int i = 0; i < S; i++) add_stats(tot, lg[i]->stats);
    g->stats = tot;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

// Address of the static scratch on `device` (which must be current): taken
// once per device with hipGetSymbolAddress and kept.  Host code never uses
// the array's own name as an address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_base[kMaxDevices] = {};

int scratch_base(int device, char **out) {
    if (device < 0 || device >= kMaxDevices) return fail(MFBC_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_base[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MFBC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_base[device] = (char *)p;
    }
    *out = g_scratch_base[device];
    return MFBC_OK;
}

// The workspace of `ncg` groups carved from `base` (same arrays and sizes as
// ensure_workspace allocates, each 256-byte aligned).
void carve_workspace(const mfbc_graph *g, int ncg, char *base, Workspace &ws) {
    ws = Workspace{};
    const int groups = ws_groups(ncg);
    size_t off = 0;
    ws_arrays(g, ws, groups, [&](auto *&p, size_t count) {
        p = (std::remove_reference_t<decltype(p)>)(base + off);
        off = align256(off + std::max<size_t>(count, 1) * sizeof(*p));
    });
    ws.ncg = groups;
    ws.external = true;
}

// Swaps a graph's own workspace out for the duration of a call and back.
struct WorkspaceSwap {
    mfbc_graph *g;
    Workspace saved;
    explicit WorkspaceSwap(mfbc_graph *gr) : g(gr), saved(gr->ws) { g->ws = Workspace{}; }
    ~WorkspaceSwap() { g->ws = saved; }
};

}  // namespace

extern "C" {

const char *mfbc_last_error(void) { return g_err.c_str(); }

int mfbc_load_graph(int32_t n, int64_t n_arcs, const int64_t *h_row_ptr, const int32_t *h_col_idx,
                    const int32_t *h_weight, uint32_t flags, void *hip_stream, mfbc_graph **out) {
    if (!out) return fail(MFBC_EINVAL, "out is NULL");
    *out = nullptr;
    const uint32_t kind = flags & ~(uint32_t)MFBC_KEEP_ORDER;
    if (kind != MFBC_UNDIRECTED && kind != MFBC_DIRECTED)
        return fail(MFBC_EINVAL, "flags must be MFBC_UNDIRECTED or MFBC_DIRECTED "
                                 "(optionally | MFBC_KEEP_ORDER)");
    int32_t maxw = 1;
    {
        std::string msg;
        const int vrc = validate_csr(n, n_arcs, h_row_ptr, h_col_idx, h_weight, &maxw, msg);
        if (vrc) return fail(vrc, msg);
    }
    std::vector<int64_t> rpt;
    std::vector<int32_t> colt, wt;
    build_transpose(n, n_arcs, h_row_ptr, h_col_idx, h_weight, rpt, colt, wt);
    const bool directed = kind == MFBC_DIRECTED;
    if (!directed && !is_symmetric(n, n_arcs, h_row_ptr, h_col_idx, h_weight, rpt, colt, wt))
        return fail(MFBC_EINVAL, "undirected graph must have a symmetric CSR with equal weights");
    // device numbering: out-arcs (rp_o, col_o, w_o) and in-arcs (rpt, colt, wt)
    const int64_t *rp_o = h_row_ptr;
    const int32_t *col_o = h_col_idx, *w_o = h_weight;
    std::vector<int32_t> perm, iperm;
    std::vector<int64_t> rpo;
    std::vector<int32_t> colo, wo;
    if (!(flags & MFBC_KEEP_ORDER)) {
        degree_order(n, n_arcs, h_row_ptr, h_col_idx, perm, iperm);
        relabel_reverse(n, n_arcs, h_row_ptr, h_col_idx, h_weight, perm, iperm, rpt, colt, wt);
        if (directed) {
            build_transpose(n, n_arcs, rpt.data(), colt.data(), h_weight ? wt.data() : nullptr,
                            rpo, colo, wo);
            rp_o = rpo.data();
            col_o = colo.data();
            w_o = h_weight ? wo.data() : nullptr;
        } else {
            rp_o = rpt.data();
            col_o = colt.data();
            w_o = h_weight ? wt.data() : nullptr;
        }
    }
    mfbc_graph *g = new (std::nothrow) mfbc_graph();
    if (!g) return fail(MFBC_ENOMEM, "host allocation failed");
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(MFBC_EDEVICE, "no HIP device");
    }
    g->n = n;
    g->arcs = n_arcs;
    g->maxw = maxw;
    g->weighted = h_weight != nullptr;
    g->directed = directed;
    // packed frontier tuples: weight bits for (n - 1) * max weight (+1 so that
    // no tuple equals the all-ones "absent" marker), the rest for multiplicities
    g->mb = 32 - bits_for((int64_t)(n - 1) * maxw + 1);
    int rc = upload_csr(n, n_arcs, rp_o, col_o, w_o, maxw, g->out);
    if (!rc) {
        if (directed)
            rc = upload_csr(n, n_arcs, rpt.data(), colt.data(), h_weight ? wt.data() : nullptr,
                            maxw, g->in);
        else
            g->in = g->out;
    }
    if (!rc && !perm.empty()) {
        if (!(rc = dalloc(&g->perm, (size_t)n))) {
            if (hipMemcpy(g->perm, perm.data(), (size_t)n * sizeof(int32_t),
                          hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(MFBC_EDEVICE, "copy of the vertex order failed");
            g->h_perm = std::move(perm);
        }
    }
    g->params = default_params(n, n_arcs);
    g->h_rp_out.assign(rp_o, rp_o + (size_t)n + 1);
    g->h_rp_in = directed ? rpt : g->h_rp_out;
    if (!rc && hipHostMalloc((void **)&g->h_ctr,
                             sizeof(unsigned long long) * kCounterRing * 4 * kCounterSlots) !=
                   hipSuccess) {
        g->h_ctr = nullptr;
        rc = fail(MFBC_ENOMEM, "pinned host allocation failed");
    }
    if (!rc) rc = upload_plan(n, g->h_rp_out.data(), g->params, g->plan_out);
    if (!rc) rc = upload_plan(n, g->h_rp_in.data(), g->params, g->plan_in);
    if (rc) {
        free_graph_memory(g);
        delete g;
        return rc;
    }
    (void)hip_stream;
    *out = g;
    return MFBC_OK;
}

int mfbc_free_graph(mfbc_graph *g) {
    if (!g) return MFBC_OK;
    // a live server holds the graph's CSR, plan and its own back pointer
    if (g->servers > 0)
        return fail(MFBC_EINVAL, "the graph has live servers (mfbc_server_create); free them "
                                 "before the graph");
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();
    free_graph_memory(g);
    delete g;
    return MFBC_OK;
}

int mfbc_forward(mfbc_graph *g, const int32_t *d_sources, int32_t nb, int32_t *d_dist,
                 double *d_sigma, int32_t *h_products, void *hip_stream) {
    return forward_impl(g, d_sources, nb, d_dist, d_sigma, false, nullptr, nullptr, nullptr, 0,
                        h_products, hip_stream);
}

int mfbc_fixpoint(mfbc_graph *g, int32_t op, const int32_t *d_sources, int32_t nb,
                  void *d_out, int32_t *h_products, void *hip_stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (!mono_op_known(op)) return fail(MFBC_EINVAL, "unknown operation");
    if (nb < 1) return fail(MFBC_EINVAL, "nb must be >= 1");
    if (!d_out) return fail(MFBC_EINVAL, "output pointer is NULL");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = check_sources(g, d_sources, nb, s);
    if (rc) return rc;
    const int ncg = (nb + kWave - 1) / kWave;
    if ((rc = ensure_workspace(g, ncg))) return rc;
    g->stats = mfbc_stats{};
    launch_set_sources(g, ncg, nb, d_sources, s);
    launch_mono_init(g, op, ncg, nb, s);
    const double arc_bytes = g->weighted && op != MFBC_OP_BFS ? 8.0 : 4.0;
    mfbc_stats &st = g->stats;
    int64_t prev = nb;
    int j = 0, last = 0;
    // windows of products with one counter read-back each, as in MFBF
    while (!last) {
        if (j > g->n + 1) return fail(MFBC_EDEVICE, "fixpoint products did not converge");
        for (int i = 0; i < kWindow; i++) launch_mono_product(g, op, ncg, j + 1 + i, s, window_events(g, i, true));
        if ((rc = read_ring(g, s))) return rc;
        for (int i = 0; i < kWindow; i++) {
            const int jj = j + 1 + i;
            st.fwd_pull_launches++;
            add_times(g, i, &st.fwd_pull_ms, &st.fwd_merge_ms, true);
            if (last) continue;
            const Counts c = ring_counts(g, jj);
            st.fwd_entries += c.produced;
            st.fwd_outputs += c.outputs;
            st.fwd_active_vertices += c.active_vertices;
            st.fwd_active_arcs += c.active_arcs;
            // adjacency of the active rows, frontier values read once, T read
            // where a candidate arrived, T and the next frontier written per entry
            st.fwd_alg_bytes += 8.0 * c.active_vertices + arc_bytes * c.active_arcs +
                                4.0 * (double)(prev + c.outputs) + 8.0 * (double)c.produced;
            prev = c.produced;
            if (c.produced == 0) last = jj;
        }
        j += kWindow;
    }
    j = last;
    st.fwd_products = j;
    st.batches = 1;
    if (h_products) *h_products = j;
    // 4-byte values whatever their type: the tile export copies them as int32
    launch_export_tiles_i32(g, ncg, nb, g->ws.tdist, (int32_t *)d_out, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

int mfbc_forward_trace(mfbc_graph *g, const int32_t *d_sources, int32_t nb, int32_t *d_dist,
                       double *d_sigma, uint64_t *d_fbits, int32_t max_products, int64_t *h_nnz,
                       int64_t *h_relax, int32_t *h_products, void *hip_stream) {
    return forward_impl(g, d_sources, nb, d_dist, d_sigma, true, d_fbits, h_nnz, h_relax,
                        max_products, h_products, hip_stream);
}

int mfbc_backward(mfbc_graph *g, const int32_t *d_sources, int32_t nb, const int32_t *d_dist,
                  const double *d_sigma, double *d_delta, int32_t *h_products, void *hip_stream) {
    return backward_impl(g, d_sources, nb, d_dist, d_sigma, d_delta, nullptr, h_products,
                         hip_stream);
}

int mfbc_backward_trace(mfbc_graph *g, const int32_t *d_sources, int32_t nb, const int32_t *d_dist,
                        const double *d_sigma, double *d_delta, int32_t *d_step,
                        int32_t *h_products, void *hip_stream) {
    if (!d_step) return fail(MFBC_EINVAL, "d_step is NULL");
    return backward_impl(g, d_sources, nb, d_dist, d_sigma, d_delta, d_step, h_products,
                         hip_stream);
}

int mfbc_bc(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources, int32_t batch,
            double *d_bc, void *hip_stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (n_sources < 0) return fail(MFBC_EINVAL, "n_sources must be >= 0");
    if (batch < 1) return fail(MFBC_EINVAL, "batch must be >= 1");
    if (!d_bc) return fail(MFBC_EINVAL, "d_bc is NULL");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = check_sources(g, d_sources, n_sources, s);
    if (rc) return rc;
    const int ncg = bc_groups(n_sources, batch);
    const int S = lanes_for(g, (n_sources + batch - 1) / batch, ncg);
    if (S > 1) return bc_lanes(g, d_sources, n_sources, batch, ncg, S, d_bc, s);
    if ((rc = ensure_workspace(g, ncg))) return rc;
    return bc_batches(g, d_sources, n_sources, batch, ncg, d_bc, s);
}

int mfbc_bc_requests(mfbc_graph *g, const int32_t *d_sources, const int64_t *h_first,
                     int32_t n_requests, int32_t batch, double *const *h_out, void *hip_stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (n_requests < 0) return fail(MFBC_EINVAL, "n_requests must be >= 0");
    if (batch < kWave || batch % kWave || batch > kWave * kMaxBatchGroups)
        return fail(MFBC_EINVAL, "batch must be a multiple of 64 in [64, 4096]");
    if (n_requests == 0) return MFBC_OK;
    if (!h_first || !h_out) return fail(MFBC_EINVAL, "h_first or h_out is NULL");
    if (h_first[0] != 0) return fail(MFBC_EINVAL, "h_first[0] must be 0");
    for (int32_t r = 0; r < n_requests; r++) {
        if (h_first[r + 1] < h_first[r]) return fail(MFBC_EINVAL, "h_first must be non-decreasing");
        if (!h_out[r]) return fail(MFBC_EINVAL, "an output pointer is NULL");
    }
    const int64_t total = h_first[n_requests];
    if (total > 0 && !d_sources) return fail(MFBC_EINVAL, "d_sources is NULL");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = check_sources(g, d_sources, total, s);
    if (rc) return rc;
    // every request's sources in whole column groups, requests in list order
    struct Slot {
        int64_t first;
        int32_t count, req;
    };
    std::vector<Slot> slots;
    for (int32_t r = 0; r < n_requests; r++)
        for (int64_t k = h_first[r]; k < h_first[r + 1]; k += kWave)
            slots.push_back({k, (int32_t)std::min<int64_t>(kWave, h_first[r + 1] - k), r});
    for (int32_t r = 0; r < n_requests; r++) launch_zero_f64(h_out[r], (size_t)g->n, s);
    const int G = batch / kWave;
    const int ncg = (int)std::min<size_t>((size_t)G, slots.size());
    g->stats = mfbc_stats{};
    if (ncg > 0 && (rc = ensure_workspace(g, ncg))) return rc;
    for (size_t b0 = 0; b0 < slots.size(); b0 += (size_t)G) {
        const int bcg = (int)std::min<size_t>((size_t)G, slots.size() - b0);
        GroupSpans sp{};
        GroupOuts o{};
        for (int cg = 0; cg < bcg; cg++) {
            sp.first[cg] = slots[b0 + cg].first;
            sp.count[cg] = slots[b0 + cg].count;
            o.out[cg] = h_out[slots[b0 + cg].req];
        }
        launch_set_sources_spans(g, bcg, d_sources, sp, s);
        launch_lambda_zero(g, bcg, s);
        // padding columns (source -1) seed nothing and reach nothing
        if ((rc = run_forward(g, bcg, bcg * kWave, false, nullptr, nullptr, nullptr, 0, nullptr, s)))
            return rc;
        if ((rc = run_backward(g, bcg, bcg * kWave, nullptr, s))) return rc;
        launch_lambda_add_groups(g, bcg, o, s);
        g->stats.batches++;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MFBC_OK;
}

int mfbc_set_lanes(mfbc_graph *g, int32_t lanes) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (lanes < 0 || lanes > kMaxLanes)
        return fail(MFBC_EINVAL, "lanes must be in [0, " + std::to_string(kMaxLanes) + "]");
    g->lanes = lanes;
    return MFBC_OK;
}

int mfbc_bc_noalloc(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources, int32_t batch,
                    double *d_bc, void *hip_stream) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (n_sources < 0) return fail(MFBC_EINVAL, "n_sources must be >= 0");
    if (batch < 1) return fail(MFBC_EINVAL, "batch must be >= 1");
    if (!d_bc) return fail(MFBC_EINVAL, "d_bc is NULL");
    if (n_sources > 0 && !d_sources) return fail(MFBC_EINVAL, "sources pointer is NULL");
    DeviceGuard dg(g->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncg = bc_groups(n_sources, batch);
    const size_t need = ws_bytes(g, ncg);
    if (need > kScratchBytes)
        return fail(MFBC_ENOMEM, "mfbc_bc_noalloc: this graph and batch need " + std::to_string(need) +
                                     " bytes of workspace; the static scratch holds " +
                                     std::to_string(kScratchBytes));
    char *base = nullptr;
    int rc = scratch_base(g->device, &base);
    if (rc) return rc;
    // the caller's workspace stays untouched: the batch state is carved from
    // the scratch and swapped in for the duration of the call
    WorkspaceSwap sw(g);
    carve_workspace(g, ncg, base, g->ws);
    // sources are checked on the device (no host copy of the list)
    launch_check_sources(d_sources, n_sources, g->n, g->ws.flags + 1, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(g->h_ctr, g->ws.flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*(const int32_t *)g->h_ctr != 0) return fail(MFBC_EINVAL, "a source is outside [0, n)");
    return bc_batches(g, d_sources, n_sources, batch, ncg, d_bc, s);
}

int mfbc_set_plan(mfbc_graph *g, int32_t run_arcs, int32_t run_verts, int32_t heavy,
                  int32_t slice) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (run_verts > 64) return fail(MFBC_EINVAL, "run_verts must be <= 64");
    // a run's arcs are addressed with 32-bit offsets in the kernels
    if (run_arcs > (1 << 24) || heavy > (1 << 24) || slice > (1 << 24))
        return fail(MFBC_EINVAL, "run_arcs, heavy and slice must be <= 2^24");
    // a server sizes its hub partials by the plan it was created with
    if (g->servers > 0)
        return fail(MFBC_EINVAL, "the graph has live servers (mfbc_server_create); free them "
                                 "before changing its plan");
    DeviceGuard dg(g->device);
    TaskParams p = default_params(g->n, g->arcs);
    if (run_arcs > 0) p.run_arcs = run_arcs;
    if (run_verts > 0) p.run_verts = run_verts;
    if (heavy > 0) p.heavy = heavy;
    if (slice > 0) p.slice = slice;
    HIP_TRY(hipDeviceSynchronize());
    const int32_t old_slots = std::max(g->plan_in.nslots, g->plan_out.nslots);
    g->params = p;
    int rc = upload_plan(g->n, g->h_rp_out.data(), p, g->plan_out);
    if (!rc) rc = upload_plan(g->n, g->h_rp_in.data(), p, g->plan_in);
    if (rc) return rc;
    // the partial buffers are sized by the slot count: regrow on next use
    if (std::max(g->plan_in.nslots, g->plan_out.nslots) > old_slots) {
        free_workspace(g->ws);
        for (auto *sh : g->shadow)
            if (sh) free_workspace(sh->ws);
    }
    return MFBC_OK;
}

int mfbc_enable_timing(mfbc_graph *g, int enable) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (enable < 0 || enable > 2) return fail(MFBC_EINVAL, "enable must be 0, 1 or 2");
    DeviceGuard dg(g->device);
    if (enable && !g->ev[0]) {
        for (auto &e : g->ev) HIP_TRY(hipEventCreate(&e));
        for (int i = 0; i < 3 * kWindow; i++) g->ev_pull[i] = i % 3 == 2 ? nullptr : g->ev[i];
    }
    g->timing = g->ev[0] != nullptr ? enable : 0;
    return MFBC_OK;
}

int mfbc_bc_many(int32_t n_graphs, mfbc_graph *const *graphs, const int32_t *const *d_sources,
                 const int64_t *h_n_sources, double *const *d_bc, const mfbc_many_config *config,
                 mfbc_stats *h_stats, void *hip_stream) {
    if (n_graphs < 0) return fail(MFBC_EINVAL, "n_graphs must be >= 0");
    if (n_graphs == 0) return MFBC_OK;
    if (!graphs || !d_sources || !h_n_sources || !d_bc)
        return fail(MFBC_EINVAL, "array argument is NULL");
    const int dev = graphs[0] ? graphs[0]->device : 0;
    std::vector<mfbc_graph *> gs((size_t)n_graphs);
    std::vector<const int32_t *> src((size_t)n_graphs);
    std::vector<int64_t> ns((size_t)n_graphs);
    std::vector<double *> out((size_t)n_graphs);
    for (int32_t i = 0; i < n_graphs; i++) {
        if (!graphs[i]) return fail(MFBC_EINVAL, "graph " + std::to_string(i) + " is NULL");
        if (graphs[i]->device != dev) return fail(MFBC_EINVAL, "graphs live on different devices");
        if (h_n_sources[i] < 0) return fail(MFBC_EINVAL, "negative source count");
        if (!d_bc[i]) return fail(MFBC_EINVAL, "output " + std::to_string(i) + " is NULL");
        gs[(size_t)i] = graphs[i];
        src[(size_t)i] = d_sources[i];
        ns[(size_t)i] = h_n_sources[i];
        out[(size_t)i] = d_bc[i];
    }
    int block_threads = config && config->block_threads ? config->block_threads : 512;
    if (block_threads != 256 && block_threads != 512)
        return fail(MFBC_EINVAL, "block_threads must be 256 or 512");
    const int job_width = config && config->job_width ? config->job_width : kWave;
    if (job_width != kWave && job_width != 2 * kWave)
        return fail(MFBC_EINVAL, "job_width must be 64 or 128");
    const int w = job_width / kWave;
    DeviceGuard dg(dev);
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    for (int32_t i = 0; i < n_graphs; i++)
        if ((rc = check_sources(gs[(size_t)i], src[(size_t)i], ns[(size_t)i], s))) return rc;
    int blocks = config && config->blocks > 0 ? config->blocks : 0;
    if (blocks == 0) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        blocks = (2048 / block_threads) * prop.multiProcessorCount;   // 8 waves per SIMD
    }
    int n_max = 1, slots_max = 1;
    int64_t arcs_max = 1;
    for (auto *g : gs) {
        n_max = std::max(n_max, g->n);
        slots_max = std::max({slots_max, g->plan_in.nslots, g->plan_out.nslots});
        arcs_max = std::max<int64_t>(arcs_max, g->arcs);
    }
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const size_t slot = many_slot_bytes(n_max, slots_max, arcs_max, w);
    ManyWorkspace &ws = many_workspace(dev);
    // half of the memory free or already held by the workspace: the same cap
    // on every call, so a first call runs with the block count of later ones
    const size_t budget = (free_b + ws_scratch_bytes(ws)) / 2;
    const int cap = (int)std::max<size_t>(1, budget / std::max<size_t>(slot, 1));
    blocks = std::min(blocks, cap);
    // one persistent launch per arc encoding (unweighted, packed, separate)
    unsigned long long tot[2] = {0, 0};
    for (int mode = 0; mode < 3; mode++) {
        std::vector<mfbc_graph *> g2;
        std::vector<const int32_t *> s2;
        std::vector<int64_t> n2;
        std::vector<double *> o2;
        for (size_t i = 0; i < gs.size(); i++) {
            const Csr &c = gs[i]->in;
            const int m = c.w == nullptr ? 0 : (c.pk ? 1 : 2);
            if (m != mode) continue;
            g2.push_back(gs[i]);
            s2.push_back(src[i]);
            n2.push_back(ns[i]);
            o2.push_back(out[i]);
        }
        if (g2.empty()) continue;
        unsigned long long st[2] = {0, 0};
        int32_t flags[2] = {0, 0};
        std::string err;
        rc = launch_bc_many(g2, s2, n2, o2, block_threads, blocks, w, s, ws, st, flags, err);
        if (rc) return fail(rc, err);
        if (flags[1]) return fail(MFBC_EDEVICE, "products did not converge");
        if (flags[0]) return fail(MFBC_EOVERFLOW, "a shortest-path count overflowed binary64");
        tot[0] += st[0];
        tot[1] += st[1];
    }
    if (h_stats) {
        *h_stats = mfbc_stats{};
        h_stats->fwd_products = (int64_t)tot[0];
        h_stats->bwd_products = (int64_t)tot[1];
    }
    return MFBC_OK;
}

int mfbc_get_stats(const mfbc_graph *g, mfbc_stats *out) {
    if (!g || !out) return fail(MFBC_EINVAL, "NULL argument");
    *out = g->stats;
    return MFBC_OK;
}

int mfbc_graph_info(const mfbc_graph *g, int32_t *n, int64_t *n_arcs, int32_t *max_weight) {
    if (!g) return fail(MFBC_EINVAL, "graph handle is NULL");
    if (n) *n = g->n;
    if (n_arcs) *n_arcs = g->arcs;
    if (max_weight) *max_weight = g->maxw;
    return MFBC_OK;
}

}  // extern "C"
