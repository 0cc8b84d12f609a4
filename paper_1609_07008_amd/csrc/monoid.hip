// Generic monoid relaxation to a fixpoint over maximal frontiers.
//
// The paper's product C = A (+).f B (a commutative monoid (+) over the
// outputs and an action f of an arc on an input entry, Section 3) iterated
// the way Algorithm 1 iterates it: a batch of sources, T the best value per
// (source, vertex) so far, and each product relaxing only the entries that
// improved in the previous one.  Here with values in int32 and (+) = min:
//   OP 0  single-source shortest paths   f(a, w) = a + w
//   OP 1  breadth-first hop levels       f(a, w) = a + 1
// Unlike MFBF no multiplicity is carried, so a tie does not re-enter the
// frontier: an entry joins frontier j exactly when product j lowered it.
//
// Same data layout and work decomposition as the MFBF forward product:
// [cg][v][64] tiles (lane = source column), per-column-group vertex bitmaps,
// runs of light rows and slices of hub rows merged in slice order; batches
// of two or more groups run on pairs of them, the frontier values of groups
// 2p and 2p+1 interleaved per lane (one 8-byte gather for both) with one
// bitmap per pair, as in the forward product.
#include "products.h"

namespace mfbc {
namespace {

struct MonoArgs {
    const Task *tasks;
    const Hub *hubs;
    int ntasks, nhubs, nslots, ncg, n, nwords;
    const int64_t *rp;
    ArcSrc arcs;
    const uint32_t *abits;     // frontier F_{j-1}: [cg][nwords] bitmaps
    const int32_t *fval;       //   values [cg][n][64], kInf = absent
    int32_t *tval;             // T
    uint32_t *abits_n;         // frontier F_j
    int32_t *fval_n;
    int32_t *pd;               // hub partials [cg][slots][64]
    unsigned long long *ctr;   // counter slots of product j
    const unsigned long long *prev_ctr;  // nullable: those of product j-1 (live_prev)
    uint32_t *clear_bits;      // merge: F_{j-1}'s bitmaps, ncg planes
    unsigned long long *clear_ctr;
    int nwide;                 // pairs of groups (paired layout), 0: one group per wave
};

template <int OP>
__device__ __forceinline__ int mono_act(int x, int w) {
    return OP == 0 ? x + w : x + 1;
}

// T := min(T, best) at (v, cg); an entry that went down joins the next
// frontier.  Returns the lane mask of new frontier entries.
__device__ __forceinline__ uint64_t mono_finalize(const MonoArgs &a, size_t cgv, int v, int best,
                                                  int td, int lane, unsigned long long &outs) {
    const bool has = best != kInf;
    const uint64_t hm = ballot(has);
    outs += __popcll(hm);
    if (!hm) return 0;
    const size_t idx = (cgv + (size_t)v) * kWave + lane;
    const bool keep = has && best < td;
    if (keep) a.tval[idx] = best;
    const uint64_t bits = ballot(keep);
    if (bits) a.fval_n[idx] = keep ? best : kInf;
    return bits;
}

// One pull task: active arcs taken U at a time across owners, with the T row
// of each owner that starts in the batch loaded in the same round trip (as
// in the MFBF forward product).
template <int OP, int AM, int U = 8>
__device__ __forceinline__ void mono_task(const MonoArgs &a, int cg, int t,
                                          unsigned long long &produced, unsigned long long &outs) {
    const int lane = threadIdx.x & (kWave - 1);
    const Task *tp = a.tasks + t;
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const size_t cgv = (size_t)cg * (size_t)a.n;
    const int32_t *Fv = a.fval + cgv * kWave;
    const int32_t *Td = a.tval + (cgv + (size_t)v0) * kWave + lane;
    const uint32_t *Ab = a.abits + (size_t)cg * a.nwords;
    const int64_t rend = (hub < 0 && v0 + lane < v1) ? a.rp[v0 + lane + 1] : INT64_MAX;
    int cur = -1, best = kInf, td = kInf;
    uint64_t run_act = 0;
    int un = 0, wn = 1;
    if (e0 + lane < e1) load_arc<AM>(a.arcs, e0 + lane, un, wn);
    for (int64_t e = e0; e < e1; e += kWave) {
        const int64_t my = e + lane;
        const int u = un, wt = wn;
        const bool act = my < e1 && ((Ab[u >> 5] >> (u & 31)) & 1u);
        if (my + kWave < e1) load_arc<AM>(a.arcs, my + kWave, un, wn);
        uint64_t am = ballot(act);
        while (am) {
            int ow[U], wk[U], tk[U], tn[U];
            int prev = cur;
#pragma unroll
            for (int k = 0; k < U; k++) {
                const int j = am ? __ffsll((unsigned long long)am) - 1 : -1;
                am &= am - 1;
                ow[k] = -1;
                wk[k] = 0;
                tk[k] = kInf;
                tn[k] = kInf;
                if (j >= 0) {
                    const int uk = rdlane(u, j);
                    wk[k] = AM ? rdlane(wt, j) : 1;
                    tk[k] = Fv[(size_t)uk * kWave + lane];
                    ow[k] = __popcll(ballot(rend <= e + j));
                    if (hub < 0 && ow[k] != prev) tn[k] = Td[(size_t)ow[k] * kWave];
                    prev = ow[k];
                }
            }
#pragma unroll
            for (int k = 0; k < U; k++) {
                if (ow[k] >= 0) {
                    if (ow[k] != cur) {
                        if (cur >= 0 && hub < 0) {
                            const uint64_t b = mono_finalize(a, cgv, v0 + cur, best, td, lane, outs);
                            produced += __popcll(b);
                            if (b) run_act |= 1ull << cur;
                        }
                        cur = ow[k];
                        best = kInf;
                        td = tn[k];
                    }
                    if (tk[k] != kInf) best = min(best, mono_act<OP>(tk[k], wk[k]));
                }
            }
        }
    }
    if (hub < 0) {
        if (cur >= 0) {
            const uint64_t b = mono_finalize(a, cgv, v0 + cur, best, td, lane, outs);
            produced += __popcll(b);
            if (b) run_act |= 1ull << cur;
        }
        if (lane == 0 && run_act) or_run_bits(a.abits_n + (size_t)cg * a.nwords, v0, run_act);
    } else {
        a.pd[((size_t)cg * a.nslots + part) * kWave + lane] = best;
    }
}

// Combine the slices of hub row h (min is order-free) and finish it.
__device__ __forceinline__ void mono_hub(const MonoArgs &a, int cg, int h,
                                         unsigned long long &produced, unsigned long long &outs) {
    const int lane = threadIdx.x & (kWave - 1);
    const Hub *hp = a.hubs + h;
    const int v = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
    const size_t cgv = (size_t)cg * (size_t)a.n;
    int best = kInf;
    for (int p = first; p < first + np; p++)
        best = min(best, a.pd[((size_t)cg * a.nslots + p) * kWave + lane]);
    const int td = a.tval[(cgv + (size_t)v) * kWave + lane];
    const uint64_t b = mono_finalize(a, cgv, v, best, td, lane, outs);
    produced += __popcll(b);
    if (b && lane == 0) atomicOr(a.abits_n + (size_t)cg * a.nwords + (v >> 5), 1u << (v & 31));
}

// Paired form: groups 2q and 2q+1 at once (frontier values interleaved per
// lane); T keeps the one-group layout.  Returns the lanes in the next
// frontier in either group.
__device__ __forceinline__ uint64_t mono_finalize2(const MonoArgs &a, int q, int v, int b0, int b1,
                                                   int t0, int t1, int lane, unsigned long long &outs,
                                                   unsigned long long &produced) {
    const uint64_t h0 = ballot(b0 != kInf), h1 = ballot(b1 != kInf);
    outs += __popcll(h0) + __popcll(h1);
    if (!(h0 | h1)) return 0;
    const size_t n = (size_t)a.n;
    const size_t i0 = ((size_t)(2 * q) * n + (size_t)v) * kWave + lane, i1 = i0 + n * kWave;
    const bool k0 = b0 != kInf && b0 < t0, k1 = b1 != kInf && b1 < t1;
    if (k0) a.tval[i0] = b0;
    if (k1) a.tval[i1] = b1;
    const uint64_t m0 = ballot(k0), m1 = ballot(k1);
    produced += __popcll(m0) + __popcll(m1);
    if (m0 | m1)
        ((int2 *)a.fval_n)[((size_t)q * n + (size_t)v) * kWave + lane] =
            make_int2(k0 ? b0 : kInf, k1 ? b1 : kInf);
    return m0 | m1;
}

template <int OP, int AM, int U = 4>
__device__ __forceinline__ void mono_task2(const MonoArgs &a, int q, int t, unsigned long long &produced,
                                           unsigned long long &outs) {
    const int lane = threadIdx.x & (kWave - 1);
    const Task *tp = a.tasks + t;
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const size_t n = (size_t)a.n;
    const int2 *Fv = (const int2 *)a.fval + (size_t)q * n * kWave;
    const int32_t *Td0 = a.tval + ((size_t)(2 * q) * n + (size_t)v0) * kWave + lane;
    const int32_t *Td1 = Td0 + n * kWave;
    const uint32_t *Ab = a.abits + (size_t)q * a.nwords;
    const int64_t rend = (hub < 0 && v0 + lane < v1) ? a.rp[v0 + lane + 1] : INT64_MAX;
    int cur = -1, best0 = kInf, best1 = kInf, td0 = kInf, td1 = kInf;
    uint64_t run_act = 0;
    auto close = [&](int o) {
        if (mono_finalize2(a, q, v0 + o, best0, best1, td0, td1, lane, outs, produced))
            run_act |= 1ull << o;
    };
    int un = 0, wn = 1;
    if (e0 + lane < e1) load_arc<AM>(a.arcs, e0 + lane, un, wn);
    for (int64_t e = e0; e < e1; e += kWave) {
        const int64_t my = e + lane;
        const int u = un, wt = wn;
        const bool act = my < e1 && ((Ab[u >> 5] >> (u & 31)) & 1u);
        if (my + kWave < e1) load_arc<AM>(a.arcs, my + kWave, un, wn);
        uint64_t am = ballot(act);
        while (am) {
            int ow[U], wk[U], tn0[U], tn1[U];
            int2 tk[U];
            int prev = cur;
#pragma unroll
            for (int k = 0; k < U; k++) {
                const int j = am ? __ffsll((unsigned long long)am) - 1 : -1;
                am &= am - 1;
                ow[k] = -1;
                wk[k] = 0;
                tk[k] = make_int2(kInf, kInf);
                tn0[k] = kInf;
                tn1[k] = kInf;
                if (j >= 0) {
                    const int uk = rdlane(u, j);
                    wk[k] = AM ? rdlane(wt, j) : 1;
                    tk[k] = Fv[(size_t)uk * kWave + lane];
                    ow[k] = __popcll(ballot(rend <= e + j));
                    if (hub < 0 && ow[k] != prev) {
                        tn0[k] = Td0[(size_t)ow[k] * kWave];
                        tn1[k] = Td1[(size_t)ow[k] * kWave];
                    }
                    prev = ow[k];
                }
            }
#pragma unroll
            for (int k = 0; k < U; k++) {
                if (ow[k] >= 0) {
                    if (ow[k] != cur) {
                        if (cur >= 0 && hub < 0) close(cur);
                        cur = ow[k];
                        best0 = best1 = kInf;
                        td0 = tn0[k];
                        td1 = tn1[k];
                    }
                    if (tk[k].x != kInf) best0 = min(best0, mono_act<OP>(tk[k].x, wk[k]));
                    if (tk[k].y != kInf) best1 = min(best1, mono_act<OP>(tk[k].y, wk[k]));
                }
            }
        }
    }
    if (hub < 0) {
        if (cur >= 0) close(cur);
        if (lane == 0 && run_act) or_run_bits(a.abits_n + (size_t)q * a.nwords, v0, run_act);
    } else {
        const size_t p0 = ((size_t)(2 * q) * a.nslots + part) * kWave + lane;
        a.pd[p0] = best0;
        a.pd[p0 + (size_t)a.nslots * kWave] = best1;
    }
}

__device__ __forceinline__ void mono_hub2(const MonoArgs &a, int q, int h, unsigned long long &produced,
                                          unsigned long long &outs) {
    const int lane = threadIdx.x & (kWave - 1);
    const Hub *hp = a.hubs + h;
    const int v = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
    const size_t n = (size_t)a.n;
    int b0 = kInf, b1 = kInf;
    // four slices' partials in flight (min is order-free)
    for (int p = first; p < first + np; p += 4) {
        int d0[4], d1[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            d0[k] = kInf;
            d1[k] = kInf;
            if (p + k < first + np) {
                const size_t p0 = ((size_t)(2 * q) * a.nslots + p + k) * kWave + lane;
                d0[k] = a.pd[p0];
                d1[k] = a.pd[p0 + (size_t)a.nslots * kWave];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            b0 = min(b0, d0[k]);
            b1 = min(b1, d1[k]);
        }
    }
    const size_t i0 = ((size_t)(2 * q) * n + (size_t)v) * kWave + lane;
    const int t0 = b0 != kInf ? a.tval[i0] : kInf;
    const int t1 = b1 != kInf ? a.tval[i0 + n * kWave] : kInf;
    const uint64_t b = mono_finalize2(a, q, v, b0, b1, t0, t1, lane, outs, produced);
    if (b && lane == 0) atomicOr(a.abits_n + (size_t)q * a.nwords + (v >> 5), 1u << (v & 31));
}

template <int OP, int AM>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_mono_pull2(MonoArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int q = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (q < a.nwide) mono_task2<OP, AM>(a, q, wid - q * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

__global__ __launch_bounds__(kBlock) void k_mono_merge2(MonoArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.nwide, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int q = a.nhubs ? wid / a.nhubs : a.nwide;
    if (q < a.nwide) mono_hub2(a, q, wid - q * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

// Seeds of the paired layout: a source's pair row starts with every lane of
// both groups absent, then its own lane carries 0.
__global__ void k_mono_seed_rows2(const int32_t *src, int nb, int n, int2 *fval) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const size_t row = ((size_t)(c / (2 * kWave)) * n + src[c]) * kWave;
    for (int l = 0; l < kWave; l++) fval[row + l] = make_int2(kInf, kInf);
}

__global__ void k_mono_seed2(const int32_t *src, int nb, int n, int nwords, int32_t *tval,
                             int32_t *fval, uint32_t *abits) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int v = src[c];
    const int cg = c / kWave, lane = c % kWave, q = cg >> 1;
    tval[((size_t)cg * n + v) * kWave + lane] = 0;
    fval[(((size_t)q * n + v) * kWave + lane) * 2 + (cg & 1)] = 0;
    atomicOr(abits + (size_t)q * nwords + (v >> 5), 1u << (v & 31));
}

template <int OP, int AM>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_mono_pull(MonoArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (cg < a.ncg) mono_task<OP, AM>(a, cg, wid - cg * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

__global__ __launch_bounds__(kBlock) void k_mono_merge(MonoArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.ncg, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) mono_hub(a, cg, wid - cg * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

// T = INF everywhere, both bitmaps and all counters cleared.
__global__ void k_mono_fill(int32_t *tval, size_t total, uint32_t *ab0, uint32_t *ab1, size_t nab,
                            unsigned long long *ctr, int nctr) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < total; i += stride) tval[i] = kInf;
    for (size_t i = t0; i < nab; i += stride) {
        ab0[i] = 0u;
        ab1[i] = 0u;
    }
    for (size_t i = t0; i < (size_t)nctr; i += stride) ctr[i] = 0ull;
}

// The sources' rows of the first frontier start with every lane absent ...
__global__ void k_mono_seed_rows(const int32_t *src, int nb, int n, int32_t *fval) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const size_t row = ((size_t)(c / kWave) * n + src[c]) * kWave;
    for (int l = 0; l < kWave; l++) fval[row + l] = kInf;
}

// ... then T(s, s) = 0 and the first frontier is {s} carrying 0.
__global__ void k_mono_seed(const int32_t *src, int nb, int n, int nwords, int32_t *tval,
                            int32_t *fval, uint32_t *abits) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int v = src[c];
    const int cg = c / kWave, lane = c % kWave;
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    tval[idx] = 0;
    fval[idx] = 0;
    atomicOr(abits + (size_t)cg * nwords + (v >> 5), 1u << (v & 31));
}

inline int nblk(size_t work, int per, int cap = 0x7fffffff) {
    size_t b = (work + per - 1) / per;
    return (int)std::max<size_t>(1, std::min<size_t>(b, (size_t)cap));
}

ArcSrc mono_arcs(const Csr &c) {
    ArcSrc r{};
    r.col = c.col;
    r.w = c.w;
    r.pk = c.pk;
    r.cb = c.cb;
    r.cmask = c.cb >= 32 ? 0xffffffffu : ((1u << c.cb) - 1u);
    return r;
}

int mono_mode(const Csr &c) { return c.w == nullptr ? 0 : (c.pk ? 1 : 2); }

template <int OP>
void launch_pull(int mode, int grid, hipStream_t s, const MonoArgs &a) {
    if (a.nwide) {
        switch (mode) {
            case 0: hipLaunchKernelGGL((k_mono_pull2<OP, 0>), dim3(grid), dim3(kBlock), 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_mono_pull2<OP, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
            default: hipLaunchKernelGGL((k_mono_pull2<OP, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
        }
        return;
    }
    switch (mode) {
        case 0: hipLaunchKernelGGL((k_mono_pull<OP, 0>), dim3(grid), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_mono_pull<OP, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_mono_pull<OP, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
    }
}

// Batches of two or more groups run on pairs (the workspace holds an even
// number of groups).
int mono_pairs(int ncg) { return ncg >= 2 ? (ncg + 1) / 2 : 0; }

}  // namespace

void launch_mono_init(mfbc_graph *g, int ncg, int nb, hipStream_t s) {
    Workspace &ws = g->ws;
    const size_t total = (size_t)ncg * g->n * kWave;
    const int nwords = (g->n + 31) / 32;
    hipLaunchKernelGGL(k_mono_fill, dim3(nblk(total, 256, 65536)), dim3(256), 0, s, ws.tdist, total,
                       ws.abits[0], ws.abits[1], (size_t)ncg * nwords, ws.counters,
                       kCounterRing * 4 * kCounterSlots);
    if (mono_pairs(ncg)) {
        hipLaunchKernelGGL(k_mono_seed_rows2, dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                           (int2 *)ws.fdist[0]);
        hipLaunchKernelGGL(k_mono_seed2, dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                           nwords, ws.tdist, ws.fdist[0], ws.abits[0]);
        return;
    }
    hipLaunchKernelGGL(k_mono_seed_rows, dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                       ws.fdist[0]);
    hipLaunchKernelGGL(k_mono_seed, dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n, nwords,
                       ws.tdist, ws.fdist[0], ws.abits[0]);
}

void launch_mono_product(mfbc_graph *g, int op, int ncg, int j, hipStream_t s, hipEvent_t *ev) {
    Workspace &ws = g->ws;
    const int b = (j - 1) & 1;      // buffer holding F_{j-1}
    MonoArgs a{};
    a.tasks = g->plan_in.tasks;
    a.hubs = g->plan_in.hubs;
    a.ntasks = g->plan_in.ntasks;
    a.nhubs = g->plan_in.nhubs;
    a.nslots = g->plan_in.nslots;
    a.ncg = ncg;
    a.n = g->n;
    a.nwords = (g->n + 31) / 32;
    a.rp = g->in.rp;
    a.arcs = mono_arcs(g->in);
    a.abits = ws.abits[b];
    a.fval = ws.fdist[b];
    a.tval = ws.tdist;
    a.abits_n = ws.abits[b ^ 1];
    a.fval_n = ws.fdist[b ^ 1];
    a.pd = ws.pd;
    a.ctr = ws.counters + (size_t)(j % kCounterRing) * 4 * kCounterSlots;
    a.prev_ctr = j > 1 ? ws.counters + (size_t)((j - 1) % kCounterRing) * 4 * kCounterSlots : nullptr;
    a.clear_bits = ws.abits[b];
    a.clear_ctr = ws.counters + (size_t)((j + 1) % kCounterRing) * 4 * kCounterSlots;
    a.nwide = mono_pairs(ncg);
    const int waves_per_task = a.nwide ? a.nwide : ncg;
    if (ev) (void)hipEventRecord(ev[0], s);
    const int grid = nblk((size_t)a.ntasks * waves_per_task, kWavesPerBlock);
    if (op == 0) launch_pull<0>(mono_mode(g->in), grid, s, a);
    else launch_pull<1>(mono_mode(g->in), grid, s, a);
    if (ev) (void)hipEventRecord(ev[1], s);
    const int mgrid = std::max(nblk((size_t)a.nhubs * waves_per_task, kWavesPerBlock),
                               nblk((size_t)a.nwords, kBlock, 1024));
    if (a.nwide)
        hipLaunchKernelGGL(k_mono_merge2, dim3(mgrid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_mono_merge, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev) (void)hipEventRecord(ev[2], s);
}

}  // namespace mfbc
