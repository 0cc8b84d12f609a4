// Generic monoid relaxation to a fixpoint over maximal frontiers.
//
// The paper's product C = A (+).f B (a commutative monoid (+) over the
// outputs and an action f of an arc on an input entry, Section 3) iterated
// the way Algorithm 1 iterates it: a batch of sources, T the best value per
// (source, vertex) so far, and each product relaxing only the entries that
// improved in the previous one.  The algebra is a template parameter (Op:
// the value type, (+), f, the identity and the seed); the product itself is
// the generic pull product of pull.h -- the same function MFBF's forward
// product instantiates -- with MonoPull as its policy.  Instances:
//   SSSP    int32, (+) = min, f(a, w) = a + w          shortest-path distances
//   BFS     int32, (+) = min, f(a, w) = a + 1          hop levels
//   Widest  int32, (+) = max, f(a, w) = min(a, w)      bottleneck capacities
//   Resist  float, (+) = min, f(a, w) = a + 1/w        least sum of 1/w along a
//           path (binary32, every operation IEEE round-to-nearest)
// Unlike MFBF no multiplicity is carried, so a tie does not re-enter the
// frontier: an entry joins frontier j exactly when product j improved it
// (strictly, in the order of (+)).
//
// Same data layout and work decomposition as the MFBF forward product:
// [cg][v][64] tiles (lane = source column), per-column-group vertex bitmaps,
// runs of light rows and slices of hub rows merged in slice order; batches
// of two or more groups run on pairs of them, the frontier values of groups
// 2p and 2p+1 interleaved per lane (one 8-byte gather for both) with one
// bitmap per pair, as in the forward product.  Values are 4 bytes, stored in
// the workspace's int32 tiles whatever their type.
#include <type_traits>

#include "products.h"

namespace mfbc {
namespace {

struct MonoArgs {
    const Task *tasks;
    const Hub *hubs;
    int ntasks, nhubs, nslots, ncg, n, nwords;
    const int64_t *rp;
    ArcSrc arcs;
    const uint32_t *abits;     // frontier F_{j-1}: [plane][nwords] bitmaps
    const void *fval;          //   values [cg][n][64] (or pairs [q][n][64][2]), absent = Op::absent()
    void *tval;                // T, [cg][n][64]
    uint32_t *abits_n;         // frontier F_j
    void *fval_n;
    void *pd;                  // hub partials [cg][slots][64]
    unsigned long long *ctr;   // counter slots of product j
    const unsigned long long *prev_ctr;  // nullable: those of product j-1 (live_prev)
    uint32_t *clear_bits;      // merge: F_{j-1}'s bitmaps
    unsigned long long *clear_ctr;
    int nwide;                 // pairs of groups (paired layout), 0: one group per wave
};

// ------------------------------------------------------------------ algebras
struct OpSssp {
    using V = int32_t;
    __device__ static V absent() { return kInf; }
    __device__ static V seed() { return 0; }
    __device__ static V act(V x, int w) { return x + w; }
    __device__ static V plus(V x, V y) { return min(x, y); }
    __device__ static bool better(V x, V y) { return x < y; }
};

struct OpBfs {
    using V = int32_t;
    __device__ static V absent() { return kInf; }
    __device__ static V seed() { return 0; }
    __device__ static V act(V x, int) { return x + 1; }
    __device__ static V plus(V x, V y) { return min(x, y); }
    __device__ static bool better(V x, V y) { return x < y; }
};

// widths are >= 1, so 0 is "no path"; the source's own width is unbounded
struct OpWidest {
    using V = int32_t;
    __device__ static V absent() { return 0; }
    __device__ static V seed() { return kInf; }
    __device__ static V act(V x, int w) { return min(x, w); }
    __device__ static V plus(V x, V y) { return max(x, y); }
    __device__ static bool better(V x, V y) { return x > y; }
};

struct OpResist {
    using V = float;
    __device__ static V absent() { return __builtin_inff(); }
    __device__ static V seed() { return 0.0f; }
    // IEEE division (the library is built without fast-math) and one add:
    // no fused multiply-add can form
    __device__ static V act(V x, int w) { return x + 1.0f / (float)w; }
    __device__ static V plus(V x, V y) { return y < x ? y : x; }
    __device__ static bool better(V x, V y) { return x < y; }
};

template <class V, int W> struct Lanes;      // W values of one lane in one load
template <> struct Lanes<int32_t, 1> { using T = int32_t; };
template <> struct Lanes<int32_t, 2> { using T = int2; };
template <> struct Lanes<float, 1> { using T = float; };
template <> struct Lanes<float, 2> { using T = float2; };

// ------------------------------------------------------------------ the policy
// The fixpoint's product as an instance of pull_task / pull_hub: W column
// groups per lane (1, or 2 in the paired layout), T in the one-group layout.
template <class Op, int AM_, int W>
struct MonoPull : PullDefaults {
    using V = typename Op::V;
    using L = typename Lanes<V, W>::T;
    static_assert(sizeof(V) == 4, "values live in the 4-byte workspace tiles");
    static constexpr int AM = AM_;
    static constexpr int U = W == 1 ? 8 : 4;
    static constexpr int H = W == 1 ? 1 : 4;
    struct Row { V x[W]; };
    using Acc = Row;
    using Own = Row;
    const MonoArgs &a;
    const int q, lane;
    const size_t n, plane;
    const L *Fv;
    V *Tv;
    const uint32_t *bits;
    uint32_t *bits_n;
    unsigned long long &produced, &outs;

    __device__ __forceinline__ MonoPull(const MonoArgs &a_, int q_, unsigned long long &pr,
                                        unsigned long long &ou)
        : a(a_), q(q_), lane(threadIdx.x & (kWave - 1)), n((size_t)a_.n),
          plane((size_t)a_.n * kWave), Fv((const L *)a_.fval + (size_t)q_ * plane),
          Tv((V *)a_.tval + (size_t)W * q_ * plane), bits(a_.abits + (size_t)q_ * a_.nwords),
          bits_n(a_.abits_n + (size_t)q_ * a_.nwords), produced(pr), outs(ou) {}

    __device__ __forceinline__ static Row fill(V v) {
        Row r;
#pragma unroll
        for (int c = 0; c < W; c++) r.x[c] = v;
        return r;
    }
    __device__ __forceinline__ Row absent() const { return fill(Op::absent()); }
    __device__ __forceinline__ Own none() const { return fill(Op::absent()); }
    __device__ __forceinline__ Row gather(int u, const Tag &, int) const {
        const L v = Fv[(size_t)u * kWave + lane];
        Row r;
        __builtin_memcpy(r.x, &v, sizeof(v));
        return r;
    }
    __device__ __forceinline__ Own own(int v0, int o) const {
        Own t;
#pragma unroll
        for (int c = 0; c < W; c++) t.x[c] = Tv[(size_t)c * plane + ((size_t)v0 + (size_t)o) * kWave + lane];
        return t;
    }
    __device__ __forceinline__ void batch(Row (&)[U], const int (&)[U]) const {}
    __device__ __forceinline__ void reset(Acc &x) const { x = fill(Op::absent()); }
    __device__ __forceinline__ void fold(Acc &x, const Row &r, int w, int) const {
#pragma unroll
        for (int c = 0; c < W; c++)
            if (r.x[c] != Op::absent()) x.x[c] = Op::plus(x.x[c], Op::act(r.x[c], w));
    }
    // T := T (+) acc at v; an entry that improved joins the next frontier
    // (the whole row is written when any lane of any group joins).
    __device__ __forceinline__ uint64_t finish(int v, const Acc &x, const Own &t) {
        uint64_t any = 0;
#pragma unroll
        for (int c = 0; c < W; c++) {
            const uint64_t h = ballot(x.x[c] != Op::absent());
            outs += __popcll(h);
            any |= h;
        }
        if (!any) return 0;
        Row nx;
        uint64_t kept = 0;
#pragma unroll
        for (int c = 0; c < W; c++) {
            const bool keep = x.x[c] != Op::absent() && Op::better(x.x[c], t.x[c]);
            if (keep) Tv[(size_t)c * plane + (size_t)v * kWave + lane] = x.x[c];
            nx.x[c] = keep ? x.x[c] : Op::absent();
            const uint64_t b = ballot(keep);
            produced += __popcll(b);
            kept |= b;
        }
        if (kept) {
            L o;
            __builtin_memcpy(&o, nx.x, sizeof(o));
            ((L *)a.fval_n)[(size_t)q * plane + (size_t)v * kWave + lane] = o;
        }
        return kept;
    }
    __device__ __forceinline__ size_t slot(int c, int part) const {
        return ((size_t)(W * q + c) * a.nslots + part) * kWave + lane;
    }
    __device__ __forceinline__ void store(int part, const Acc &x) const {
#pragma unroll
        for (int c = 0; c < W; c++) ((V *)a.pd)[slot(c, part)] = x.x[c];
    }
    __device__ __forceinline__ Acc load(int part) const {
        Acc x;
#pragma unroll
        for (int c = 0; c < W; c++) x.x[c] = ((const V *)a.pd)[slot(c, part)];
        return x;
    }
    __device__ __forceinline__ void merge(Acc &x, const Acc &y) const {
#pragma unroll
        for (int c = 0; c < W; c++) x.x[c] = Op::plus(x.x[c], y.x[c]);
    }
    __device__ __forceinline__ uint64_t finish_hub(int v, const Acc &x) {
        Own t;
#pragma unroll
        for (int c = 0; c < W; c++)
            t.x[c] = x.x[c] != Op::absent() ? Tv[(size_t)c * plane + (size_t)v * kWave + lane]
                                            : Op::absent();
        return finish(v, x, t);
    }
};

// ------------------------------------------------------------------ kernels
template <class Op, int AM, int W>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_mono_pull(MonoArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int groups = W == 1 ? a.ncg : a.nwide;
    const int q = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (q < groups) {
        MonoPull<Op, AM, W> p(a, q, produced, outs);
        pull_task(p, a.tasks + (wid - q * a.ntasks), a.rp, a.arcs);
    }
    flush_counts(produced, outs, 0, 0, a.ctr);
}

// Hub slices of F_{j-1}'s product; also clears F_{j-1}'s bitmaps (counting
// its vertices and their arcs) and the counters of product j+1.
template <class Op, int W>
__global__ __launch_bounds__(kBlock) void k_mono_merge(MonoArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    const int groups = W == 1 ? a.ncg : a.nwide;
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, groups, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int q = a.nhubs ? wid / a.nhubs : groups;
    if (q < groups) {
        MonoPull<Op, 0, W> p(a, q, produced, outs);
        pull_hub(p, a.hubs + (wid - q * a.nhubs));
    }
    flush_counts(produced, outs, nv, na, a.ctr);
}

// T = absent everywhere, both bitmaps and all counters cleared.
template <class Op>
__global__ void k_mono_fill(typename Op::V *tval, size_t total, uint32_t *ab0, uint32_t *ab1, size_t nab,
                            unsigned long long *ctr, int nctr) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < total; i += stride) tval[i] = Op::absent();
    for (size_t i = t0; i < nab; i += stride) {
        ab0[i] = 0u;
        ab1[i] = 0u;
    }
    for (size_t i = t0; i < (size_t)nctr; i += stride) ctr[i] = 0ull;
}

// The sources' rows of the first frontier start with every lane of their
// plane absent (W groups per lane) ...
template <class Op, int W>
__global__ void k_mono_seed_rows(const int32_t *src, int nb, int n, typename Op::V *fval) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const size_t row = ((size_t)(c / (W * kWave)) * n + src[c]) * kWave * W;
    for (int l = 0; l < kWave * W; l++) fval[row + l] = Op::absent();
}

// ... then T(s, s) = the seed and the first frontier is {s} carrying it.
template <class Op, int W>
__global__ void k_mono_seed(const int32_t *src, int nb, int n, int nwords, typename Op::V *tval,
                            typename Op::V *fval, uint32_t *abits) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int v = src[c];
    const int cg = c / kWave, lane = c % kWave, q = cg / W;
    tval[((size_t)cg * n + v) * kWave + lane] = Op::seed();
    fval[(((size_t)q * n + v) * kWave + lane) * W + (cg % W)] = Op::seed();
    atomicOr(abits + (size_t)q * nwords + (v >> 5), 1u << (v & 31));
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

template <class Op, int W>
void launch_pull(int mode, int grid, hipStream_t s, const MonoArgs &a) {
    switch (mode) {
        case 0: hipLaunchKernelGGL((k_mono_pull<Op, 0, W>), dim3(grid), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_mono_pull<Op, 1, W>), dim3(grid), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_mono_pull<Op, 2, W>), dim3(grid), dim3(kBlock), 0, s, a); break;
    }
}

// Batches of two or more groups run on pairs (the workspace holds an even
// number of groups).
int mono_pairs(int ncg) { return ncg >= 2 ? (ncg + 1) / 2 : 0; }

template <class Op>
void mono_init(mfbc_graph *g, int ncg, int nb, hipStream_t s) {
    using V = typename Op::V;
    Workspace &ws = g->ws;
    const size_t total = (size_t)ncg * g->n * kWave;
    const int nwords = (g->n + 31) / 32;
    hipLaunchKernelGGL(k_mono_fill<Op>, dim3(nblk(total, 256, 65536)), dim3(256), 0, s, (V *)ws.tdist,
                       total, ws.abits[0], ws.abits[1], (size_t)ncg * nwords, ws.counters,
                       kCounterRing * 4 * kCounterSlots);
    if (mono_pairs(ncg)) {
        hipLaunchKernelGGL((k_mono_seed_rows<Op, 2>), dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb,
                           g->n, (V *)ws.fdist[0]);
        hipLaunchKernelGGL((k_mono_seed<Op, 2>), dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                           nwords, (V *)ws.tdist, (V *)ws.fdist[0], ws.abits[0]);
        return;
    }
    hipLaunchKernelGGL((k_mono_seed_rows<Op, 1>), dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                       (V *)ws.fdist[0]);
    hipLaunchKernelGGL((k_mono_seed<Op, 1>), dim3(nblk(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                       nwords, (V *)ws.tdist, (V *)ws.fdist[0], ws.abits[0]);
}

template <class Op>
void mono_product(mfbc_graph *g, int ncg, int j, hipStream_t s, hipEvent_t *ev) {
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
    if (a.nwide) launch_pull<Op, 2>(mono_mode(g->in), grid, s, a);
    else launch_pull<Op, 1>(mono_mode(g->in), grid, s, a);
    if (ev) (void)hipEventRecord(ev[1], s);
    const int mgrid = std::max(nblk((size_t)a.nhubs * waves_per_task, kWavesPerBlock),
                               nblk((size_t)a.nwords, kBlock, 1024));
    if (a.nwide)
        hipLaunchKernelGGL((k_mono_merge<Op, 2>), dim3(mgrid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_mono_merge<Op, 1>), dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
}

}  // namespace

bool mono_op_known(int op) {
    return op == MFBC_OP_SSSP || op == MFBC_OP_BFS || op == MFBC_OP_WIDEST || op == MFBC_OP_RESIST;
}

void launch_mono_init(mfbc_graph *g, int op, int ncg, int nb, hipStream_t s) {
    switch (op) {
        case MFBC_OP_SSSP: mono_init<OpSssp>(g, ncg, nb, s); break;
        case MFBC_OP_BFS: mono_init<OpBfs>(g, ncg, nb, s); break;
        case MFBC_OP_WIDEST: mono_init<OpWidest>(g, ncg, nb, s); break;
        default: mono_init<OpResist>(g, ncg, nb, s); break;
    }
}

void launch_mono_product(mfbc_graph *g, int op, int ncg, int j, hipStream_t s, hipEvent_t *ev) {
    switch (op) {
        case MFBC_OP_SSSP: mono_product<OpSssp>(g, ncg, j, s, ev); break;
        case MFBC_OP_BFS: mono_product<OpBfs>(g, ncg, j, s, ev); break;
        case MFBC_OP_WIDEST: mono_product<OpWidest>(g, ncg, j, s, ev); break;
        default: mono_product<OpResist>(g, ncg, j, s, ev); break;
    }
}

}  // namespace mfbc
