// Batched form: MFBC over many graphs in one persistent launch.
//
// A job is (graph, up to 64 W sources: W column groups, W = 1 or 2); each
// workgroup takes jobs from a
// device-side queue (one atomic per job) and runs the whole of Algorithm 3
// for its job -- forward products until the frontier empties, the counting
// product, backward products until the backward frontier empties -- with
// only workgroup barriers between products: no kernel launch and no host
// round trip per product, which is what dominates the per-graph launch
// sequence on graphs of a few thousand vertices.  The products are the same
// task and hub functions as the grid-wide kernels (products.h), scheduled
// over the workgroup's waves; jobs of two groups run the paired functions
// (one gather per arc for 128 columns), as the plain path does.  Each job's state lives in its workgroup's slot
// of a scratch area sized for the largest graph; each job's lambda goes to
// its own slice and the slices of a graph are summed in job order, so the
// result does not depend on which workgroup ran which job.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "products.h"

namespace mfbc {

struct GraphDesc {
    int32_t n, nwords, mb, am;        // am: arc mode of both orientations
    int32_t ntasks_in, nhubs_in, nslots_in, ntasks_out;
    int32_t nhubs_out, nslots_out, pad0, pad1;
    const int64_t *rp_in, *rp_out;
    ArcSrc arcs_in, arcs_out;
    const Task *tasks_in, *tasks_out;
    const Hub *hubs_in, *hubs_out;
    const int32_t *perm;       // caller id -> device id (nullable)
};

struct JobDesc {
    int32_t g, nsrc;
    const int32_t *src;        // device pointer to this job's first source
    int64_t lam_off;           // offset of this job's lambda slice
};

struct ManyArgs {
    const GraphDesc *graphs;
    const JobDesc *jobs;
    int32_t njobs, n_max, slots_max, pad;
    int64_t arcs_max;                // largest out-arc count: the slot's DAG masks
    unsigned int *queue;
    char *scratch;
    size_t slot_stride;
    double *lam_jobs;
    int32_t *flags;                  // [0] overflow, [1] no convergence
    unsigned long long *stats;       // [0] forward products, [1] backward products
};

namespace {

constexpr int kManyMaxThreads = 512;

__device__ __forceinline__ size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A workgroup's state for jobs of W column groups: per-(column, vertex)
// arrays [W][n_max][64] (the frontier tuples and backward lane masks in the
// paired layout when W = 2), one activity bitmap per buffer, the stored DAG
// [W][arcs].
struct Slot {
    int32_t *tdist;
    double *tsig;
    uint32_t *ftup[2];
    double *fsig[2];
    uint64_t *fbits[2];
    uint32_t *abits[2];
    int32_t *pd;
    double *pm;
    int32_t *src;
    uint64_t *dag;             // shortest-path lane mask per out-arc and group
};

template <int W>
__device__ __forceinline__ Slot carve(char *base, int n_max, int slots_max) {
    Slot s;
    const size_t nw = (size_t)n_max * kWave * W;
    const size_t words = ((size_t)n_max + 31) / 32;
    size_t off = 0;
    s.tdist = (int32_t *)(base + off); off = align256(off + nw * 4);
    s.tsig = (double *)(base + off); off = align256(off + nw * 8);
    for (int b = 0; b < 2; b++) {
        s.ftup[b] = (uint32_t *)(base + off); off = align256(off + nw * 4);
        s.fsig[b] = (double *)(base + off); off = align256(off + nw * 8);
        s.fbits[b] = (uint64_t *)(base + off); off = align256(off + (size_t)n_max * 8 * W);
        s.abits[b] = (uint32_t *)(base + off); off = align256(off + words * 4);
    }
    s.pd = (int32_t *)(base + off); off = align256(off + (size_t)slots_max * kWave * 4 * W);
    s.pm = (double *)(base + off); off = align256(off + (size_t)slots_max * kWave * 8 * W);
    s.src = (int32_t *)(base + off); off = align256(off + kWave * 4 * W);
    s.dag = (uint64_t *)(base + off);
    return s;
}

// Pointer of buffer b (0 or 1) without indexing an array by a runtime value
// (which would put the pair in scratch memory).
template <typename T>
__device__ __forceinline__ T *pick(T *const (&p)[2], int b) {
    return b ? p[1] : p[0];
}

// AM: arc encoding shared by every graph of the launch (see load_arc); W:
// column groups per job.  Eight waves per SIMD: the loop is bound by the
// latency of its dependent gathers, and more resident waves hide more of it
// than the spills (uniform state kept in VGPR lanes and a small private
// segment) cost.
template <int AM, int W>
__global__ __launch_bounds__(kManyMaxThreads) __attribute__((amdgpu_waves_per_eu(8)))
void k_bc_many(ManyArgs m) {
    constexpr int C = W * kWave;       // columns per job
    __shared__ int s_job;
    __shared__ unsigned long long s_cnt[3];
    __shared__ int32_t s_full;       // the job's tau does not fit the compact copy
    const int tid = threadIdx.x, nthr = blockDim.x;
    // wave index as a uniform (scalar) value, so the task loops stay uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwaves = nthr >> 6;
    const bool lead = (tid & (kWave - 1)) == 0;
    const Slot sl = carve<W>(m.scratch + (size_t)blockIdx.x * m.slot_stride, m.n_max, m.slots_max);
    for (;;) {
        if (tid == 0) s_job = (int)atomicAdd(m.queue, 1u);
        if (tid < 3) s_cnt[tid] = 0ull;
        __syncthreads();
        const int job = s_job;
        if (job >= m.njobs) break;
        const JobDesc jd = m.jobs[job];
        const GraphDesc gd = m.graphs[jd.g];
        const int n = gd.n, nw = gd.nwords;
        const size_t plane = (size_t)n * kWave;
        double *lam = m.lam_jobs + jd.lam_off;     // [W][n]
        // ---- Algorithm 1 initialisation: T = (INF, 0), first frontier {s}
        for (int c = tid; c < C; c += nthr)
            sl.src[c] = c < jd.nsrc ? (gd.perm ? gd.perm[jd.src[c]] : jd.src[c]) : -1;
        for (size_t i = tid; i < W * plane; i += nthr) {
            sl.tdist[i] = kInf;
            sl.tsig[i] = 0.0;
        }
        for (int i = tid; i < nw; i += nthr) {
            sl.abits[0][i] = 0u;
            sl.abits[1][i] = 0u;
        }
        for (int i = tid; i < W * n; i += nthr) lam[i] = 0.0;
        __syncthreads();
        // a source's frontier row starts with every lane of the job absent ...
        for (int c = tid; c < jd.nsrc; c += nthr) {
            const int v = sl.src[c];
            for (int l = 0; l < C; l++) sl.ftup[0][(size_t)v * C + l] = kSent;
        }
        __syncthreads();
        // ... then its own column carries (0, 1): weight 0, inline multiplicity 1
        for (int c = tid; c < jd.nsrc; c += nthr) {
            const int v = sl.src[c], g = c / kWave, lane = c % kWave;
            const size_t idx = (size_t)g * plane + (size_t)v * kWave + lane;
            sl.tdist[idx] = 0;
            sl.tsig[idx] = 1.0;
            sl.ftup[0][((size_t)v * kWave + lane) * W + g] = 1u;
            atomicOr(sl.abits[0] + (v >> 5), 1u << (v & 31));
        }
        __syncthreads();
        // ---- Algorithm 1 loop
        FwdArgs a{};
        a.tasks = gd.tasks_in;
        a.hubs = gd.hubs_in;
        a.ntasks = gd.ntasks_in;
        a.nhubs = gd.nhubs_in;
        a.nslots = gd.nslots_in;
        a.ncg = W;
        a.ncg_all = W;
        a.nwide = W == 2 ? 1 : 0;
        a.nwide_all = a.nwide;
        a.n = n;
        a.nwords = nw;
        a.mb = gd.mb;
        a.rp = gd.rp_in;
        a.arcs = gd.arcs_in;
        a.tdist = sl.tdist;
        a.tsig = sl.tsig;
        a.pd = sl.pd;
        a.pm = sl.pm;
        a.flags = m.flags;
        int j = 0;
        for (;;) {
            ++j;
            const int b = (j - 1) & 1;
            a.j = j;
            a.abits = pick(sl.abits, b);
            a.ftup = pick(sl.ftup, b);
            a.fsig = pick(sl.fsig, b);
            a.abits_n = pick(sl.abits, b ^ 1);
            a.ftup_n = pick(sl.ftup, b ^ 1);
            a.fsig_n = pick(sl.fsig, b ^ 1);
            if (tid == 0) s_cnt[(j + 1) % 3] = 0ull;
            unsigned long long produced = 0, outs = 0;
            if constexpr (W == 1) {
                for (int t = wave; t < a.ntasks; t += nwaves) fwd_task<AM, 4>(a, 0, t, produced, outs);
            } else {
                for (int t = wave; t < a.ntasks; t += nwaves) fwd_task_w<AM, W>(a, 0, t, produced, outs);
            }
            __syncthreads();
            if constexpr (W == 1) {
                for (int h = wave; h < a.nhubs; h += nwaves) fwd_hub(a, 0, h, produced, outs);
            } else {
                for (int h = wave; h < a.nhubs; h += nwaves) fwd_hub_w<W>(a, 0, h, produced, outs);
            }
            for (int i = tid; i < nw; i += nthr) pick(sl.abits, b)[i] = 0u;
            if (lead && produced) atomicAdd(&s_cnt[j % 3], produced);
            __syncthreads();
            if (s_cnt[j % 3] == 0ull) break;
            if (j > n + 1) {
                if (tid == 0) m.flags[1] = 1;
                break;
            }
        }
        __syncthreads();   // every thread has read the last forward count
        // ---- Algorithm 2: counting product, then backward products
        BwdArgs c{};
        c.tasks = gd.tasks_out;
        c.hubs = gd.hubs_out;
        c.ntasks = gd.ntasks_out;
        c.nhubs = gd.nhubs_out;
        c.nslots = gd.nslots_out;
        c.ncg = W;
        c.ncg_all = W;
        c.nwide = W == 2 ? 1 : 0;
        c.nwide_all = c.nwide;
        c.n = n;
        c.nwords = nw;
        c.rp = gd.rp_out;
        c.arcs = gd.arcs_out;
        c.src = sl.src;
        c.tdist = sl.tdist;
        c.tsig = sl.tsig;
        c.cnt = (int32_t *)sl.ftup[0];
        c.zeta = sl.fsig[0];
        c.q = sl.fsig[1];
        c.step = nullptr;          // frontier indices are not reported here
        c.lam = lam;
        c.pd = sl.pd;
        c.pm = sl.pm;
        c.dag = sl.dag;            // the counting product stores the DAG, the
        c.narcs = m.arcs_max;      // backward products read it ([W][arcs_max])
        if constexpr (W == 2) {
            // tau of both groups interleaved per lane in 16 bits a group for the
            // paired counting product, unless a finite value does not fit
            uint32_t *t2 = (uint32_t *)sl.ftup[1];
            bool big = false;
            for (size_t i = tid; i < plane; i += nthr) {
                const int x = sl.tdist[i], y = sl.tdist[plane + i];
                big |= tau16_big(x) || tau16_big(y);
                t2[i] = pack_tau16(x, y);
            }
            c.tau2 = t2;
            const int full = __syncthreads_or(big);
            if (tid == 0) s_full = full;      // read after the barrier below
            c.tau_full = &s_full;
        }
        for (int i = tid; i < nw; i += nthr) {
            sl.abits[0][i] = 0u;
            sl.abits[1][i] = 0u;
        }
        if (tid == 0) {
            s_cnt[0] = 0ull;
            s_cnt[1] = 0ull;
            s_cnt[2] = 0ull;
        }
        __syncthreads();
        int k = 0;
        for (;;) {
            const int bn = k & 1;
            c.k = k;
            c.abits = pick(sl.abits, bn ^ 1);
            c.fbits = pick(sl.fbits, bn ^ 1);
            c.abits_n = pick(sl.abits, bn);
            c.fbits_n = pick(sl.fbits, bn);
            if (tid == 0) s_cnt[(k + 1) % 3] = 0ull;
            unsigned long long produced = 0, outs = 0;
            if (k == 0) {
                if constexpr (W == 1) {
                    for (int t = wave; t < c.ntasks; t += nwaves) count_task<AM>(c, 0, t, produced);
                } else {
                    if (s_full) {
                        for (int t = wave; t < c.ntasks; t += nwaves) count_task_w<AM, false, true>(c, 0, t, produced);
                    } else {
                        for (int t = wave; t < c.ntasks; t += nwaves) count_task_w<AM, false, false>(c, 0, t, produced);
                    }
                }
            } else {
                if constexpr (W == 1) {
                    for (int t = wave; t < c.ntasks; t += nwaves) bwd_task<AM>(c, 0, t, produced, outs);
                } else {
                    for (int t = wave; t < c.ntasks; t += nwaves)
                        bwd_task_w<AM, false>(c, 0, t, produced, outs);
                }
            }
            __syncthreads();
            if (k == 0) {
                for (int h = wave; h < W * c.nhubs; h += nwaves)
                    count_hub(c, h / c.nhubs, h % c.nhubs, produced);
            } else {
                if constexpr (W == 1) {
                    for (int h = wave; h < c.nhubs; h += nwaves) bwd_hub(c, 0, h, produced, outs);
                } else {
                    for (int h = wave; h < c.nhubs; h += nwaves) bwd_hub_w(c, 0, h, produced, outs);
                }
                for (int i = tid; i < nw; i += nthr) pick(sl.abits, bn ^ 1)[i] = 0u;
            }
            if (lead && produced) atomicAdd(&s_cnt[k % 3], produced);
            __syncthreads();
            const bool done = s_cnt[k % 3] == 0ull;
            ++k;
            if (done) break;
            if (k > n + 1) {
                if (tid == 0) m.flags[1] = 1;
                break;
            }
        }
        if (tid == 0) {
            atomicAdd(m.stats + 0, (unsigned long long)j);
            atomicAdd(m.stats + 1, (unsigned long long)k);
        }
        __syncthreads();
    }
}

// lambda of graph g at caller vertex v: the job slices (W planes each)
// summed in job order.
__global__ void k_many_reduce(const double *lam_jobs, const int64_t *job_off, const int32_t *jbeg,
                              const int32_t *jcnt, const int32_t *order, int n, int w, double *out,
                              const int32_t *perm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int d = perm ? perm[v] : v;
    double t = 0.0;
    for (int i = 0; i < jcnt[0]; i++)
        for (int c = 0; c < w; c++) t += lam_jobs[job_off[order[jbeg[0] + i]] + (size_t)c * n + d];
    out[v] = t;
}

}  // namespace

// Host side -----------------------------------------------------------------

struct ManyWorkspace {
    char *scratch = nullptr;
    size_t scratch_bytes = 0;
    double *lam_jobs = nullptr;
    size_t lam_bytes = 0;
    void *meta = nullptr;
    size_t meta_bytes = 0;
};

ManyWorkspace &many_workspace(int device) {
    static std::mutex mu;
    static std::vector<ManyWorkspace *> per_device;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)per_device.size() <= device) per_device.resize((size_t)device + 1, nullptr);
    if (!per_device[(size_t)device]) per_device[(size_t)device] = new ManyWorkspace();
    return *per_device[(size_t)device];
}

static size_t host_align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t many_slot_bytes(int n_max, int slots_max, int64_t arcs_max, int w) {
    const size_t nw = (size_t)n_max * kWave * w;
    const size_t words = ((size_t)n_max + 31) / 32;
    size_t off = 0;
    off = host_align256(off + nw * 4);
    off = host_align256(off + nw * 8);
    for (int b = 0; b < 2; b++) {
        off = host_align256(off + nw * 4);
        off = host_align256(off + nw * 8);
        off = host_align256(off + (size_t)n_max * 8 * w);
        off = host_align256(off + words * 4);
    }
    off = host_align256(off + (size_t)slots_max * kWave * 4 * w);
    off = host_align256(off + (size_t)slots_max * kWave * 8 * w);
    off = host_align256(off + kWave * 4 * w);
    off = host_align256(off + (size_t)std::max<int64_t>(arcs_max, 1) * 8 * w);
    return off;
}

static ArcSrc host_arc_src(const Csr &c) {
    ArcSrc r{};
    r.col = c.col;
    r.w = c.w;
    r.pk = c.pk;
    r.cb = c.cb;
    r.cmask = c.cb >= 32 ? 0xffffffffu : ((1u << c.cb) - 1u);
    return r;
}

static int host_arc_mode(const Csr &c) { return c.w == nullptr ? 0 : (c.pk ? 1 : 2); }

int launch_bc_many(std::vector<mfbc_graph *> &graphs, const std::vector<const int32_t *> &d_src,
                   const std::vector<int64_t> &n_src, const std::vector<double *> &d_bc,
                   int block_threads, int blocks, int w, hipStream_t s, ManyWorkspace &ws,
                   unsigned long long *h_stats, int32_t *h_flags, std::string &err) {
    const int G = (int)graphs.size();
    std::vector<GraphDesc> gds((size_t)G);
    int n_max = 1, slots_max = 1;
    int64_t arcs_max = 1;
    for (int i = 0; i < G; i++) {
        mfbc_graph *g = graphs[(size_t)i];
        GraphDesc &d = gds[(size_t)i];
        d = GraphDesc{};
        d.n = g->n;
        d.nwords = (g->n + 31) / 32;
        d.mb = g->mb;
        d.am = host_arc_mode(g->in);
        if (host_arc_mode(g->out) != d.am || d.am != host_arc_mode(graphs[0]->in)) {
            err = "graphs of one launch must share one arc encoding";
            return MFBC_EINVAL;
        }
        d.ntasks_in = g->plan_in.ntasks;
        d.nhubs_in = g->plan_in.nhubs;
        d.nslots_in = g->plan_in.nslots;
        d.ntasks_out = g->plan_out.ntasks;
        d.nhubs_out = g->plan_out.nhubs;
        d.nslots_out = g->plan_out.nslots;
        d.rp_in = g->in.rp;
        d.rp_out = g->out.rp;
        d.arcs_in = host_arc_src(g->in);
        d.arcs_out = host_arc_src(g->out);
        d.tasks_in = g->plan_in.tasks;
        d.tasks_out = g->plan_out.tasks;
        d.hubs_in = g->plan_in.hubs;
        d.hubs_out = g->plan_out.hubs;
        d.perm = g->perm;
        n_max = std::max(n_max, g->n);
        slots_max = std::max({slots_max, g->plan_in.nslots, g->plan_out.nslots});
        arcs_max = std::max<int64_t>(arcs_max, g->arcs);
    }
    // jobs: 64 w sources each; scheduled largest first (longest-processing-time
    // order) so that small jobs fill in at the end
    const int per_job = kWave * w;
    std::vector<JobDesc> jobs;
    std::vector<double> cost;
    int64_t lam_total = 0;
    for (int i = 0; i < G; i++) {
        const double c = (double)graphs[(size_t)i]->n * (double)(graphs[(size_t)i]->arcs + 1);
        for (int64_t b0 = 0; b0 < n_src[(size_t)i]; b0 += per_job) {
            JobDesc jd{};
            jd.g = i;
            jd.nsrc = (int32_t)std::min<int64_t>(per_job, n_src[(size_t)i] - b0);
            jd.src = d_src[(size_t)i] + b0;
            jd.lam_off = lam_total;
            lam_total += (int64_t)graphs[(size_t)i]->n * w;
            jobs.push_back(jd);
            cost.push_back(c);
        }
    }
    std::vector<int32_t> order(jobs.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return cost[(size_t)x] > cost[(size_t)y]; });
    std::vector<JobDesc> sorted(jobs.size());
    for (size_t i = 0; i < order.size(); i++) sorted[i] = jobs[(size_t)order[i]];
    // reduction order: for each graph, its jobs in source order
    std::vector<int64_t> job_off(jobs.size());
    for (size_t i = 0; i < jobs.size(); i++) job_off[i] = jobs[i].lam_off;
    std::vector<int32_t> jbeg((size_t)G), jcnt((size_t)G), jidx;
    for (int i = 0; i < G; i++) {
        jbeg[(size_t)i] = (int32_t)jidx.size();
        for (size_t q = 0; q < jobs.size(); q++)
            if (jobs[q].g == i) jidx.push_back((int32_t)q);
        jcnt[(size_t)i] = (int32_t)jidx.size() - jbeg[(size_t)i];
    }
    const int njobs = (int)jobs.size();
    blocks = std::max(1, std::min(blocks, std::max(njobs, 1)));
    const size_t slot = many_slot_bytes(n_max, slots_max, arcs_max, w);
    const size_t need_scratch = slot * (size_t)blocks;
    const size_t need_lam = (size_t)std::max<int64_t>(lam_total, 1) * sizeof(double);
    // metadata block: graphs, jobs, queue, flags, stats, offsets
    size_t moff = 0;
    const size_t o_graphs = moff; moff = host_align256(moff + gds.size() * sizeof(GraphDesc));
    const size_t o_jobs = moff; moff = host_align256(moff + std::max<size_t>(1, sorted.size()) * sizeof(JobDesc));
    const size_t o_queue = moff; moff = host_align256(moff + 16);
    const size_t o_flags = moff; moff = host_align256(moff + 16);
    const size_t o_stats = moff; moff = host_align256(moff + 16);
    const size_t o_joff = moff; moff = host_align256(moff + std::max<size_t>(1, job_off.size()) * 8);
    const size_t o_jidx = moff; moff = host_align256(moff + std::max<size_t>(1, jidx.size()) * 4);
    const size_t o_jbeg = moff; moff = host_align256(moff + (size_t)G * 4);
    const size_t o_jcnt = moff; moff = host_align256(moff + (size_t)G * 4);
    auto grow = [&](void **p, size_t &have, size_t need) -> int {
        if (have >= need) return MFBC_OK;
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        have = 0;
        if (hipMalloc(p, need) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            err = "device allocation of " + std::to_string(need) + " bytes failed";
            return MFBC_ENOMEM;
        }
        have = need;
        return MFBC_OK;
    };
    int rc;
    if ((rc = grow((void **)&ws.scratch, ws.scratch_bytes, need_scratch))) return rc;
    if ((rc = grow((void **)&ws.lam_jobs, ws.lam_bytes, need_lam))) return rc;
    if ((rc = grow(&ws.meta, ws.meta_bytes, moff))) return rc;
    char *meta = (char *)ws.meta;
    std::vector<char> h(moff, 0);
    memcpy(h.data() + o_graphs, gds.data(), gds.size() * sizeof(GraphDesc));
    if (!sorted.empty()) memcpy(h.data() + o_jobs, sorted.data(), sorted.size() * sizeof(JobDesc));
    if (!job_off.empty()) memcpy(h.data() + o_joff, job_off.data(), job_off.size() * 8);
    if (!jidx.empty()) memcpy(h.data() + o_jidx, jidx.data(), jidx.size() * 4);
    memcpy(h.data() + o_jbeg, jbeg.data(), (size_t)G * 4);
    memcpy(h.data() + o_jcnt, jcnt.data(), (size_t)G * 4);
    if (hipMemcpyAsync(meta, h.data(), moff, hipMemcpyHostToDevice, s) != hipSuccess) {
        err = "metadata upload failed";
        return MFBC_EDEVICE;
    }
    ManyArgs m{};
    m.graphs = (const GraphDesc *)(meta + o_graphs);
    m.jobs = (const JobDesc *)(meta + o_jobs);
    m.njobs = njobs;
    m.n_max = n_max;
    m.slots_max = slots_max;
    m.arcs_max = arcs_max;
    m.queue = (unsigned int *)(meta + o_queue);
    m.scratch = ws.scratch;
    m.slot_stride = slot;
    m.lam_jobs = ws.lam_jobs;
    m.flags = (int32_t *)(meta + o_flags);
    m.stats = (unsigned long long *)(meta + o_stats);
    if (njobs > 0) {
        const int key = gds[0].am * 2 + (w == 2);
        switch (key) {
            case 0: hipLaunchKernelGGL((k_bc_many<0, 1>), dim3(blocks), dim3(block_threads), 0, s, m); break;
            case 1: hipLaunchKernelGGL((k_bc_many<0, 2>), dim3(blocks), dim3(block_threads), 0, s, m); break;
            case 2: hipLaunchKernelGGL((k_bc_many<1, 1>), dim3(blocks), dim3(block_threads), 0, s, m); break;
            case 3: hipLaunchKernelGGL((k_bc_many<1, 2>), dim3(blocks), dim3(block_threads), 0, s, m); break;
            case 4: hipLaunchKernelGGL((k_bc_many<2, 1>), dim3(blocks), dim3(block_threads), 0, s, m); break;
            default: hipLaunchKernelGGL((k_bc_many<2, 2>), dim3(blocks), dim3(block_threads), 0, s, m); break;
        }
    }
    for (int i = 0; i < G; i++) {
        const int n = graphs[(size_t)i]->n;
        hipLaunchKernelGGL(k_many_reduce, dim3((n + 255) / 256), dim3(256), 0, s, ws.lam_jobs,
                           (const int64_t *)(meta + o_joff), (const int32_t *)(meta + o_jbeg) + i,
                           (const int32_t *)(meta + o_jcnt) + i, (const int32_t *)(meta + o_jidx),
                           n, w, d_bc[(size_t)i], (const int32_t *)graphs[(size_t)i]->perm);
    }
    if (hipGetLastError() != hipSuccess) {
        err = "kernel launch failed";
        return MFBC_EDEVICE;
    }
    if (hipMemcpyAsync(h_stats, meta + o_stats, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_flags, meta + o_flags, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        err = "batched launch failed";
        return MFBC_EDEVICE;
    }
    return MFBC_OK;
}

}  // namespace mfbc

namespace mfbc {
size_t ws_scratch_bytes_impl(const ManyWorkspace &ws) { return ws.scratch_bytes; }
}  // namespace mfbc
