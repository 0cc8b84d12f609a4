// Device-side building blocks of the MFBC products, shared by the
// grid-wide kernels (kernels.hip, server.hip) and the persistent
// multi-graph kernel (batched.hip).  Each product is cut into tasks (Task: a
// run of light rows or a slice of a hub row) processed by one wave for one
// column group or a pair of them, plus a per-hub merge in fixed slice order;
// the callers decide how tasks are scheduled (one grid per product, or a
// workgroup looping over them).  The forward and backward products are
// policies of the generic pull product of pull.h; the counting product and
// the per-entry finish steps are written out here.
#pragma once

#include "pull.h"

namespace mfbc {
namespace {


// Sum of a per-lane double over the wave in a fixed butterfly order.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Counters of one product, kCounterSlots-wide arrays (spread to avoid a
// single hot address): [0] frontier entries produced, [1] output entries
// that received a candidate, [2] active vertices read, [3] arcs of their rows.
// c0 and c1 are wave-uniform (every lane holds the wave's count; lane 0's
// is used), c2 and c3 are per-thread.  Block-level sum, then one atomic per
// array.
__device__ __forceinline__ void flush_counts(unsigned long long c0, unsigned long long c1,
                                             unsigned long long c2, unsigned long long c3,
                                             unsigned long long *ctr) {
    __shared__ unsigned long long s_cnt[4][kWavesPerBlock];
    const bool first = (threadIdx.x & (kWave - 1)) == 0;
    unsigned long long v[4] = {first ? c0 : 0ull, first ? c1 : 0ull, c2, c3};
#pragma unroll
    for (int k = 0; k < 4; k++) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) s_cnt[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long t = 0;
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; i++) t += s_cnt[threadIdx.x][i];
        if (t) atomicAdd(ctr + threadIdx.x * kCounterSlots + (blockIdx.x & (kCounterSlots - 1)), t);
    }
}

// Whether the product before this one produced any frontier entry: the
// first counter array of its slot (kCounterSlots partial sums written by
// flush_counts and by its merge) holds a nonzero value.  The host may
// enqueue several products before reading their counters; a product whose
// predecessor found nothing has an empty frontier to read, so every wave of
// it returns at once (the test reads the same words in every wave, so whole
// workgroups take the same branch).  nullptr: always run.
__device__ __forceinline__ bool live_prev(const unsigned long long *prev) {
    if (!prev) return true;
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long x = lane < kCounterSlots ? prev[lane] : 0ull;
    return ballot(x != 0ull) != 0ull;
}

// Clear `planes` vertex bitmaps of `words` words each while counting the
// vertices set in any of them and the arcs of their rows.
__device__ __forceinline__ void clear_and_count(uint32_t *bits, int words, int planes,
                                                const int64_t *rp, unsigned long long &nv,
                                                unsigned long long &na) {
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = gtid; i < words; i += gridDim.x * blockDim.x) {
        uint32_t w = 0u;
        for (int p = 0; p < planes; p++) {
            const uint32_t x = bits[(size_t)p * words + i];
            if (x) {
                w |= x;
                bits[(size_t)p * words + i] = 0u;
            }
        }
        if (w) {
            nv += __popc(w);
            // the arcs of a run of consecutive vertices: one row-pointer difference
            const int64_t *r = rp + (size_t)i * 32;
            while (w) {
                const int b0 = __ffs(w) - 1;
                const uint32_t from = w >> b0;
                const int len = ~from ? __ffs(~from) - 1 : 32 - b0;
                na += (unsigned long long)(r[b0 + len] - r[b0]);
                w &= ~(uint32_t)(((1ull << len) - 1ull) << b0);
            }
        }
    }
}


// Record the columns of group cg that produced frontier entries (one atomic
// per wave, spread over 32 copies that the host ORs together).
__device__ __forceinline__ void flush_colmask(unsigned long long *colmask, int ncg, int cg,
                                              uint64_t any) {
    if (colmask && any && (threadIdx.x & (kWave - 1)) == 0)
        atomicOr(colmask + (size_t)(blockIdx.x & 31) * ncg + cg, (unsigned long long)any);
}

// ===================================================================== forward
//
// Frontier tuples are packed into 32 bits: (weight << mb) | m, where the
// multiplicity m is stored inline when 1 <= m < 2^mb and m = 0 means "read
// the binary64 multiplicity from the escape array".  mb is chosen per graph
// from the largest possible frontier weight, (n - 1) * max weight (a frontier
// entry is a least-weight walk no heavier than any shorter one, hence a simple
// path).  kSent marks a lane that is not in the frontier.  A row of 64 lanes
// is 256 B; with integer weights drawn from a wide range almost every
// multiplicity is small, so the 8-byte escape is rarely read.
constexpr uint32_t kSent = 0xffffffffu;

struct FwdArgs {
    const Task *tasks;
    const Hub *hubs;
    int ntasks, nhubs, nslots, ncg, n, j, nwords;
    int mb;                    // inline multiplicity bits
    const int64_t *rp;
    ArcSrc arcs;
    const uint32_t *abits;     // frontier F_{j-1}: [cg][nwords] activity bitmaps
    const uint32_t *ftup;      //   packed tuples [cg][n][64]
    const double *fsig;        //   escaped multiplicities
    int32_t *tdist;            // T
    double *tsig;
    uint32_t *abits_n;         // frontier F_j
    uint32_t *ftup_n;
    double *fsig_n;
    int32_t *pd;               // hub partials
    double *pm;
    unsigned long long *ctr;   // counter slots of product j
    const unsigned long long *prev_ctr;  // nullable: counter slots of product j-1 (see live_prev)
    int32_t *flags;
    uint32_t *clear_bits;      // merge: bitmaps to clear (F_{j-1}'s), ncg planes
    unsigned long long *clear_ctr;  // merge: counter slots of product j+1
    unsigned long long *colmask;    // nullable: [32][ncg_all] columns that produced entries
    const int32_t *cglist;     // nullable: the ncg column groups of this launch (else 0..ncg-1)
    int ncg_all;               // column groups of the state (strides of colmask, bitmap planes)
    int nwide;                 // wide layout: groups of 2 column groups (0: one per wave)
    int nwide_all;             //   wide groups of the state (bitmap planes)
};

// T := T (+) G at one entry (idx = (cg, v, lane)) given its candidate
// (bd, bm); returns the packed tuple of the next frontier, kSent if the
// entry is not in it (no candidate, or a heavier one).  `tdin` as below.
__device__ __forceinline__ uint32_t fwd_update(const FwdArgs &a, size_t idx, int bd, double bm,
                                               int tdin);

// T := T (+) G at (v, cg); writes the next frontier row.  Returns the lane
// mask of the frontier entries produced.
// `tdin`: T's weight at (v, lane) if the caller loaded it already (it must
// have, for every owner that received a candidate), else kLoadTd.
constexpr int kLoadTd = -1;

__device__ __forceinline__ uint64_t fwd_finalize(const FwdArgs &a, size_t cgv, int v, int bd,
                                                 double bm, int tdin, int lane,
                                                 unsigned long long &outs) {
    uint64_t bits = 0;
    const uint64_t hm = ballot(bd != kInf);
    outs += __popcll(hm);
    if (hm) {
        const size_t idx = (cgv + (size_t)v) * kWave + lane;
        const uint32_t t = fwd_update(a, idx, bd, bm, tdin);
        bits = ballot(t != kSent);
        if (bits) a.ftup_n[idx] = t;
    }
    return bits;
}

__device__ __forceinline__ uint32_t fwd_update(const FwdArgs &a, size_t idx, int bd, double bm,
                                               int tdin) {
    if (bd == kInf) return kSent;
    const int td = tdin == kLoadTd ? a.tdist[idx] : tdin;
    if (bd < td) {
        a.tdist[idx] = bd;
        a.tsig[idx] = bm;
        if (__builtin_isinf(bm)) a.flags[0] = 1;
    } else if (bd == td) {
        const double s = a.tsig[idx] + bm;
        a.tsig[idx] = s;
        if (__builtin_isinf(s)) a.flags[0] = 1;
    } else {
        return kSent;
    }
    const double mmax = (double)((1u << a.mb) - 1u);
    const uint32_t ms = bm <= mmax ? (uint32_t)bm : 0u;
    if (ms == 0u) a.fsig_n[idx] = bm;
    return ((uint32_t)bd << a.mb) | ms;
}

// Active arcs per batch and whether a batch's escaped multiplicities are
// read together up front: with weights drawn from a wide range escapes are
// rare and are read lazily, only where they count (leaving registers for a
// larger batch); unweighted graphs tie often and escape often.
template <int AM> constexpr int kFwdBatch = AM == 0 ? 4 : 6;
template <int AM> constexpr bool kFwdEscBatch = AM == 0;

// ===================================================================== forward, wide
//
// The plain path runs the forward product on W = 2 column groups at once: the frontier rows of groups Wq .. Wq+W-1 are interleaved ([q][v][64]
// x W x 32 bits, one 4W-byte entry per lane), so a lane holds W columns and
// one load instruction gathers the frontier row of all W groups.  A gather's
// cost is set by its instruction more than by its bytes (64-lane loads of
// 256 B, 512 B and 1 KB issue at about the same rate from L2), so W groups
// per wave divide the gathers, the arc loads and the activity tests of a
// product by W.  W = 4 fits only six waves per SIMD and measured no faster
// overall, so the code is written for a general W and used with W = 2.  T and the escaped multiplicities keep the one-group layout;
// the activity bitmap is per wide group (a vertex active in a column of any
// of its groups), and the writer fills every slot of a row (kSent where a
// lane is not in the frontier), so a row marked active holds valid tuples
// for all W groups.

template <int W> struct WideT;
template <> struct WideT<2> { using T = uint2; };

__device__ __forceinline__ void unpack(const uint2 &v, uint32_t (&o)[2]) {
    o[0] = v.x;
    o[1] = v.y;
}
__device__ __forceinline__ uint2 pack(const uint32_t (&o)[2]) { return make_uint2(o[0], o[1]); }

// Active arcs per batch in the wide form (W columns per lane take W times
// the registers per arc; four weighted arcs at seven waves per SIMD measured
// faster than two at eight or three at seven).
template <int AM, int W> constexpr int kFwdBatchW = AM == 0 ? 2 : 4;

// T := T (+) G at (v, Wq + c) for c < W; writes the next frontier's wide
// row.  Returns the lanes in the next frontier in any of the W groups.
// `colany[c]` collects the lanes of group c that produced entries.
template <int W>
__device__ __forceinline__ uint64_t fwd_finalize_w(const FwdArgs &a, int q, int v, const int (&bd)[W],
                                                   const double (&bm)[W], const int (&td)[W], int lane,
                                                   unsigned long long &outs, unsigned long long &produced,
                                                   uint64_t (&colany)[W]) {
    uint64_t any = 0;
#pragma unroll
    for (int c = 0; c < W; c++) {
        const uint64_t h = ballot(bd[c] != kInf);
        outs += __popcll(h);
        any |= h;
    }
    if (!any) return 0;
    const size_t n = (size_t)a.n;
    const size_t i0 = ((size_t)(W * q) * n + (size_t)v) * kWave + lane;
    uint32_t t[W];
    uint64_t kept = 0;
#pragma unroll
    for (int c = 0; c < W; c++) {
        t[c] = fwd_update(a, i0 + (size_t)c * n * kWave, bd[c], bm[c], td[c]);
        const uint64_t b = ballot(t[c] != kSent);
        produced += __popcll(b);
        kept |= b;
        colany[c] |= b;
    }
    using V = typename WideT<W>::T;
    if (kept) ((V *)a.ftup_n)[((size_t)q * n + (size_t)v) * kWave + lane] = pack(t);
    return kept;
}

// Record, per group of wide group q, the columns that produced entries.
template <int W>
__device__ __forceinline__ void flush_colmask_w(const FwdArgs &a, int q, const uint64_t (&colany)[W]) {
#pragma unroll
    for (int c = 0; c < W; c++)
        if (W * q + c < a.ncg_all) flush_colmask(a.colmask, a.ncg_all, W * q + c, colany[c]);
}

// ===================================================================== forward product
//
// MFBF's forward product as an instance of the generic pull product
// (pull_task / pull_hub): (+) is the multpaths monoid (the least weight
// wins, the multiplicities of equal weights add up), f(a, w) = (a.w + w,
// a.m), over the packed tuples of W column groups per lane: W = 1 reads the
// one-group tiles [cg][v][64], W = 2 the pair layout.  T and the escaped
// multiplicities keep the one-group layout in both.
template <int AM_, int W, int U_ = (W == 1 ? kFwdBatch<AM_> : kFwdBatchW<AM_, W>)>
struct FwdPull : PullDefaults {
    static constexpr int AM = AM_;
    static constexpr int U = U_;
    static constexpr int H = W == 1 ? 1 : 4;
    static constexpr bool kEsc = kFwdEscBatch<AM_>;
    struct RowLazy {
        uint32_t t[W];
    };
    struct RowEsc {
        uint32_t t[W];
        double em[W];          // escaped multiplicities, read with the batch
    };
    using Row = std::conditional_t<kEsc, RowEsc, RowLazy>;
    struct Acc {
        int d[W];
        double m[W];
    };
    struct Own {
        int t[W];
    };
    const FwdArgs &a;
    const int q, lane;         // the wave's column group (W = 1) or pair of groups
    const size_t n, plane;
    const uint32_t *Ft;        // frontier tuples of the wave's groups
    const double *Fm;          // escaped multiplicities, group c at Fm + c * plane
    const uint32_t *bits;
    uint32_t *bits_n;
    const uint32_t mmask;
    unsigned long long &produced, &outs;
    uint64_t colany[W];        // lanes of each group that produced entries

    __device__ __forceinline__ FwdPull(const FwdArgs &a_, int q_, unsigned long long &pr,
                                       unsigned long long &ou)
        : a(a_), q(q_), lane(threadIdx.x & (kWave - 1)), n((size_t)a_.n),
          plane((size_t)a_.n * kWave), Ft(a_.ftup + (size_t)W * q_ * plane),
          Fm(a_.fsig + (size_t)W * q_ * plane), bits(a_.abits + (size_t)q_ * a_.nwords),
          bits_n(a_.abits_n + (size_t)q_ * a_.nwords), mmask((1u << a_.mb) - 1u), produced(pr),
          outs(ou) {
#pragma unroll
        for (int c = 0; c < W; c++) colany[c] = 0;
    }
    __device__ __forceinline__ Row absent() const {
        Row r;
#pragma unroll
        for (int c = 0; c < W; c++) {
            r.t[c] = kSent;
            if constexpr (kEsc) r.em[c] = 0.0;
        }
        return r;
    }
    __device__ __forceinline__ Own none() const {
        Own o;
#pragma unroll
        for (int c = 0; c < W; c++) o.t[c] = kInf;
        return o;
    }
    __device__ __forceinline__ Row gather(int u, const Tag &, int) const {
        Row r = absent();
        if constexpr (W == 1) r.t[0] = Ft[(size_t)(uint32_t)u * kWave + lane];
        else unpack(((const typename WideT<W>::T *)Ft)[(size_t)(uint32_t)u * kWave + lane], r.t);
        return r;
    }
    __device__ __forceinline__ Own own(int v0, int o) const {
        const int32_t *Td = a.tdist + ((size_t)(W * q) * n + (size_t)v0) * kWave + lane;
        Own t;
#pragma unroll
        for (int c = 0; c < W; c++) t.t[c] = Td[(size_t)c * plane + (size_t)o * kWave];
        return t;
    }
    // escaped multiplicities of the batch, read together (rare when weights
    // are drawn from a wide range; common in unweighted graphs)
    __device__ __forceinline__ void batch(Row (&r)[U], const int (&us)[U]) const {
        if constexpr (kEsc) {
            bool esc = false;
#pragma unroll
            for (int k = 0; k < U; k++)
#pragma unroll
                for (int c = 0; c < W; c++) esc |= r[k].t[c] != kSent && (r[k].t[c] & mmask) == 0u;
            if (ballot(esc)) {
#pragma unroll
                for (int k = 0; k < U; k++)
#pragma unroll
                    for (int c = 0; c < W; c++)
                        if (r[k].t[c] != kSent && (r[k].t[c] & mmask) == 0u)
                            r[k].em[c] = Fm[(size_t)c * plane + (size_t)us[k] * kWave + lane];
            }
        }
    }
    __device__ __forceinline__ void reset(Acc &x) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            x.d[c] = kInf;
            x.m[c] = 0.0;
        }
    }
    __device__ __forceinline__ void fold(Acc &x, const Row &r, int w, int u) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            const uint32_t t = r.t[c];
            const int d = (int)(t >> a.mb) + w;
            if (t != kSent && d <= x.d[c]) {
                const uint32_t ms = t & mmask;
                double m = (double)ms;
                if (!ms) {
                    if constexpr (kEsc) m = r.em[c];
                    else m = Fm[(size_t)c * plane + (size_t)u * kWave + lane];
                }
                if (d < x.d[c]) {
                    x.d[c] = d;
                    x.m[c] = m;
                } else {
                    x.m[c] += m;
                }
            }
        }
    }
    __device__ __forceinline__ uint64_t finish(int v, const Acc &x, const Own &o) {
        if constexpr (W == 1) {
            const uint64_t b = fwd_finalize(a, (size_t)q * n, v, x.d[0], x.m[0], o.t[0], lane, outs);
            produced += __popcll(b);
            colany[0] |= b;
            return b;
        } else {
            return fwd_finalize_w<W>(a, q, v, x.d, x.m, o.t, lane, outs, produced, colany);
        }
    }
    __device__ __forceinline__ size_t slot(int c, int part) const {
        return ((size_t)(W * q + c) * a.nslots + part) * kWave + lane;
    }
    __device__ __forceinline__ void store(int part, const Acc &x) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            a.pd[slot(c, part)] = x.d[c];
            a.pm[slot(c, part)] = x.m[c];
        }
    }
    __device__ __forceinline__ Acc load(int part) const {
        Acc x;
#pragma unroll
        for (int c = 0; c < W; c++) {
            x.d[c] = a.pd[slot(c, part)];
            x.m[c] = a.pm[slot(c, part)];
        }
        return x;
    }
    __device__ __forceinline__ void merge(Acc &x, const Acc &y) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            if (y.d[c] < x.d[c]) {
                x.d[c] = y.d[c];
                x.m[c] = y.m[c];
            } else if (y.d[c] == x.d[c] && y.d[c] != kInf) {
                x.m[c] += y.m[c];
            }
        }
    }
    __device__ __forceinline__ uint64_t finish_hub(int v, const Acc &x) {
        Own o;
#pragma unroll
        for (int c = 0; c < W; c++) o.t[c] = kLoadTd;
        return finish(v, x, o);
    }
    // record, per group, the columns that produced entries (served form)
    __device__ __forceinline__ void flush() const {
        if constexpr (W == 1) flush_colmask(a.colmask, a.ncg_all, q, colany[0]);
        else if (a.colmask) flush_colmask_w<W>(a, q, colany);
    }
};

// One pull task of the forward product for column group cg.
template <int AM, int U = kFwdBatch<AM>>
__device__ __forceinline__ void fwd_task(const FwdArgs &a, int cg, int t, unsigned long long &produced,
                                         unsigned long long &outs) {
    FwdPull<AM, 1, U> p(a, cg, produced, outs);
    pull_task(p, a.tasks + t, a.rp, a.arcs);
    p.flush();
}

// Combine the slices of split row h (fixed slice order) and finish it.
// The merge kernel also clears the previous frontier's bitmaps (counting
// the vertices active in some column and their arcs) and the next
// product's counters.
__device__ __forceinline__ void fwd_hub(const FwdArgs &a, int cg, int h, unsigned long long &produced,
                                        unsigned long long &outs) {
    FwdPull<0, 1> p(a, cg, produced, outs);
    pull_hub(p, a.hubs + h);
    p.flush();
}

// The same for wide group q (W column groups per lane).
template <int AM, int W>
__device__ __forceinline__ void fwd_task_w(const FwdArgs &a, int q, int t, unsigned long long &produced,
                                           unsigned long long &outs) {
    FwdPull<AM, W> p(a, q, produced, outs);
    pull_task(p, a.tasks + t, a.rp, a.arcs);
    p.flush();
}

template <int W>
__device__ __forceinline__ void fwd_hub_w(const FwdArgs &a, int q, int h, unsigned long long &produced,
                                          unsigned long long &outs) {
    FwdPull<0, W> p(a, q, produced, outs);
    pull_hub(p, a.hubs + h);
    p.flush();
}

// ===================================================================== backward
struct BwdArgs {
    const Task *tasks;
    const Hub *hubs;
    int ntasks, nhubs, nslots, ncg, n, k, nwords;
    const int64_t *rp;         // out-arcs
    ArcSrc arcs;
    const int32_t *src;        // column -> source vertex (-1 = padding)
    const int32_t *tdist;      // tau
    const double *tsig;        // sigma
    const uint32_t *abits;     // frontier B_{k-1}: [cg][nwords] activity bitmaps
    const uint64_t *fbits;     //   lane masks [cg][n]
    uint32_t *abits_n;         // frontier B_k
    uint64_t *fbits_n;
    int32_t *cnt;              // counters (> 0 pending, -1 finished or unreachable)
    double *zeta;              // partial centrality factors
    double *q;                 // frontier values zeta + 1/sigma
    int32_t *step;             // index of the backward frontier entered
    double *lam;               // [cg][n] lambda parts
    int32_t *pd;
    double *pm;
    unsigned long long *ctr;
    const unsigned long long *prev_ctr;  // nullable: counter slots of product k-1 (live_prev)
    uint32_t *clear_bits;      // ncg planes
    unsigned long long *clear_ctr;
    unsigned long long *colmask;    // nullable: [32][ncg_all] columns that produced entries
    const uint64_t *cmask;     // counting product: nullable per-group lane mask of the
                               // columns to count (others are left untouched)
    const int32_t *cglist;     // nullable: the ncg column groups of this launch (else 0..ncg-1)
    int ncg_all;               // column groups of the state (strides of colmask, bitmap planes)
    uint64_t *dag;             // the shortest-path DAG, one lane mask per out-arc, [cg][narcs]:
    int64_t narcs;             //   written by the counting product (skipped if NULL), read by
                               //   the backward products in place of the distance test
    int nwide;                 // paired layout (plain path, two or more groups): lane masks
                               //   interleaved per pair of groups, [cg/2][n][2], and one
                               //   activity bitmap per pair; 0: one group per plane
    int nwide_all;             //   pairs of the state (bitmap planes)
    const uint32_t *tau2;      // paired counting product: tau of groups 2q, 2q+1 in 16 bits
                               //   each, one word per lane, [q][n][64] (pack_tau16)
    const int32_t *tau_full;   //   nonzero: some finite tau of the launch does not fit 16 bits
                               //   (tau2 is then not read; tdist is)
};

// Index of (cg, x) in the lane masks and plane of cg in the activity bitmaps.
__device__ __forceinline__ size_t fb_index(const BwdArgs &a, int cg, int x) {
    return a.nwide ? ((size_t)(cg >> 1) * (size_t)a.n + (size_t)x) * 2 + (cg & 1)
                   : (size_t)cg * (size_t)a.n + (size_t)x;
}
__device__ __forceinline__ int ab_plane(const BwdArgs &a, int cg) { return a.nwide ? cg >> 1 : cg; }

// Per-vertex finish of the counting product: counters, leaves, zeta = 0.
__device__ __forceinline__ uint64_t count_finalize(const BwdArgs &a, size_t cgv, int cg, int x,
                                                   int dx, int c, int lane) {
    const uint64_t mask = a.cmask ? a.cmask[cg] : ~0ull;
    const bool mine = (mask >> lane) & 1ull;
    const size_t idx = (cgv + (size_t)x) * kWave + lane;
    const bool reach = dx != kInf;
    const bool leaf = reach && c == 0;
    const bool front = mine && leaf && a.src[cg * kWave + lane] != x;
    if (mine) {
        a.cnt[idx] = (reach && c > 0) ? c : -1;
        a.zeta[idx] = 0.0;
        if (a.step) a.step[idx] = leaf ? 0 : -1;
        if (leaf) a.q[idx] = 1.0 / a.tsig[idx];
    }
    const uint64_t bits = ballot(front);
    if (lane == 0) {
        uint64_t *row = a.fbits_n + fb_index(a, cg, x);
        *row = a.cmask ? ((*row & ~mask) | bits) : bits;
    }
    return bits;
}

// One task of the counting product: for every arc x -> y the lane test
// tau(y) == tau(x) + w, eight arcs' loads in flight; the lane masks of the
// arcs that pass form the stored shortest-path DAG.
template <int AM>
__device__ __forceinline__ void count_task(const BwdArgs &a, int cg, int t, unsigned long long &produced) {
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t colany = 0;
    const Task *tp = a.tasks + t;
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const size_t cgv = (size_t)cg * (size_t)a.n;
    const int32_t *Td = a.tdist + cgv * kWave;
    uint64_t run_act = 0;
    uint64_t *Dg = a.dag ? a.dag + (size_t)cg * a.narcs : nullptr;
    const int xa = v0, xb = hub >= 0 ? v0 + 1 : v1;
    for (int x = xa; x < xb; x++) {
        const int dx = Td[(size_t)x * kWave + lane];
        // lanes outside the counting mask skip their loads (their state is kept)
        const bool reach = dx != kInf && (!a.cmask || ((a.cmask[cg] >> lane) & 1ull));
        const int64_t ea = hub >= 0 ? e0 : a.rp[x];
        const int64_t eb = hub >= 0 ? e1 : a.rp[x + 1];
        int c = 0;
        if (ballot(reach)) {
            for (int64_t e = ea; e < eb; e += kWave) {
                const int64_t my = e + lane;
                int y = 0, wt = 1;
                if (my < eb) load_arc<AM>(a.arcs, my, y, wt);
                const int cnt = (int)((eb - e) < kWave ? (eb - e) : kWave);
                uint64_t mine = 0;          // this lane's arc: its shortest-path lanes
                for (int j = 0; j < cnt; j += 8) {
                    int dy[8], wj[8];
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        dy[k] = kInf;
                        wj[k] = 0;
                        if (j + k < cnt) {
                            const int yk = rdlane(y, j + k);
                            wj[k] = AM ? rdlane(wt, j + k) : 1;
                            if (reach) dy[k] = Td[(size_t)yk * kWave + lane];
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        const bool tight = reach && dy[k] != kInf && dy[k] == dx + wj[k];
                        if (tight) c++;
                        if (Dg) {
                            const uint64_t tm = ballot(tight);
                            if (lane == j + k) mine = tm;
                        }
                    }
                }
                if (Dg && my < eb) Dg[my] = mine;
            }
        } else if (Dg) {
            // no lane reaches x: none of its arcs is on a shortest path
            for (int64_t e = ea + lane; e < eb; e += kWave) Dg[e] = 0ull;
        }
        if (hub >= 0) {
            a.pd[((size_t)cg * a.nslots + part) * kWave + lane] = c;
        } else {
            const uint64_t b = count_finalize(a, cgv, cg, x, dx, c, lane);
            produced += __popcll(b);
            colany |= b;
            if (b) run_act |= 1ull << (x - v0);
        }
    }
    if (hub < 0 && lane == 0 && run_act)
        or_run_bits(a.abits_n + (size_t)ab_plane(a, cg) * a.nwords, v0, run_act);
    flush_colmask(a.colmask, a.ncg_all, cg, colany);
}

__device__ __forceinline__ void count_hub(const BwdArgs &a, int cg, int h, unsigned long long &produced) {
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t colany = 0;
    const Hub *hp = a.hubs + h;
    const int x = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
    const size_t cgv = (size_t)cg * (size_t)a.n;
    int c = 0;
    for (int p = first; p < first + np; p++) c += a.pd[((size_t)cg * a.nslots + p) * kWave + lane];
    const int dx = a.tdist[(cgv + (size_t)x) * kWave + lane];
    const uint64_t b = count_finalize(a, cgv, cg, x, dx, c, lane);
    produced += __popcll(b);
    colany |= b;
    if (b && lane == 0)
        atomicOr(a.abits_n + (size_t)ab_plane(a, cg) * a.nwords + (x >> 5), 1u << (x & 31));
    flush_colmask(a.colmask, a.ncg_all, cg, colany);
}

// tau of a pair of column groups for the paired counting product, 16 bits
// per group in one 32-bit entry per (vertex, lane): group 2q in the low half,
// 2q+1 in the high half, kTau16Inf for an unreachable vertex.  It holds only
// when every finite distance of the launch is below kTau16Big; the producer
// raises a flag otherwise (tau16_big), and the counting product then reads
// tau from tdist.  On weighted R-MAT and Erdos-Renyi graphs (weights up to
// 255) every distance fits, and the per-arc gather moves 256 B for the pair
// instead of 512.
constexpr uint32_t kTau16Inf = 0xffffu, kTau16Big = 0xfffeu;
__device__ __forceinline__ bool tau16_big(int t) { return t != kInf && (uint32_t)t >= kTau16Big; }
__device__ __forceinline__ uint32_t tau16(int t) { return t == kInf ? kTau16Inf : (uint32_t)t & 0xffffu; }
__device__ __forceinline__ uint32_t pack_tau16(int t0, int t1) { return tau16(t0) | (tau16(t1) << 16); }
__device__ __forceinline__ int unpack_tau16(uint32_t h) { return h == kTau16Inf ? kInf : (int)h; }

// One task of the counting product for the pair of column groups q (batches
// of two or more groups): tau of both groups is read from its interleaved
// 16-bit copy (tau2), so one 4-byte gather per arc and lane serves the tests
// of both groups, where one group per wave issues a 256-B gather per arc for
// each group; the owner's tau is read in full from tdist.  Each group keeps its own counters,
// leaves and DAG masks, written in the layouts the backward products of the
// batch read (fb_index, ab_plane).  A padding group (odd group count) counts
// nothing and writes nothing.
// CM (served form): count only the lanes of a.cmask and record the columns
// that produced entries in a.colmask.  FULL: tau does not fit the compact
// copy, the gathers read tdist (two 4-byte loads per arc and lane).
template <int AM, bool CM, bool FULL>
__device__ __forceinline__ void count_task_w(const BwdArgs &a, int q, int t, unsigned long long &produced) {
    const int lane = threadIdx.x & (kWave - 1);
    const int cg0 = 2 * q;
    const bool has1 = cg0 + 1 < a.ncg_all;
    const Task *tp = a.tasks + t;
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const size_t n = (size_t)a.n;
    const uint32_t *T16 = a.tau2 + (size_t)q * n * kWave;
    const int32_t *Td0 = a.tdist + (size_t)cg0 * n * kWave;
    const int32_t *Td1 = Td0 + n * kWave;       // read only when has1
    // served form: lanes outside the counting mask skip their loads
    const bool in0 = !CM || ((a.cmask[cg0] >> lane) & 1ull);
    const bool in1 = has1 && (!CM || ((a.cmask[cg0 + 1] >> lane) & 1ull));
    uint64_t *Dg0 = a.dag + (size_t)cg0 * a.narcs;
    uint64_t *Dg1 = Dg0 + a.narcs;
    uint64_t act0 = 0, act1 = 0, any0 = 0, any1 = 0;
    const int xa = v0, xb = hub >= 0 ? v0 + 1 : v1;
    for (int x = xa; x < xb; x++) {
        int2 dx;
        dx.x = Td0[(size_t)x * kWave + lane];
        dx.y = has1 ? Td1[(size_t)x * kWave + lane] : kInf;
        const bool r0 = in0 && dx.x != kInf, r1 = in1 && dx.y != kInf;
        const int64_t ea = hub >= 0 ? e0 : a.rp[x];
        const int64_t eb = hub >= 0 ? e1 : a.rp[x + 1];
        int c0 = 0, c1 = 0;
        if (ballot(r0 || r1)) {
            for (int64_t e = ea; e < eb; e += kWave) {
                const int64_t my = e + lane;
                int y = 0, wt = 1;
                if (my < eb) load_arc<AM>(a.arcs, my, y, wt);
                const int cnt = (int)((eb - e) < kWave ? (eb - e) : kWave);
                uint64_t m0 = 0, m1 = 0;     // this lane's arc: its shortest-path lanes
                for (int j = 0; j < cnt; j += 8) {
                    int2 dy[8];
                    int wj[8];
                    if constexpr (!FULL) {
                        uint32_t h[8];
#pragma unroll
                        for (int k = 0; k < 8; k++) {
                            h[k] = kTau16Inf | (kTau16Inf << 16);
                            wj[k] = 0;
                            if (j + k < cnt) {
                                const int yk = rdlane(y, j + k);
                                wj[k] = AM ? rdlane(wt, j + k) : 1;
                                h[k] = T16[(size_t)yk * kWave + lane];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 8; k++)
                            dy[k] = make_int2(unpack_tau16(h[k] & 0xffffu), unpack_tau16(h[k] >> 16));
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; k++) {
                            dy[k] = make_int2(kInf, kInf);
                            wj[k] = 0;
                            if (j + k < cnt) {
                                const int yk = rdlane(y, j + k);
                                wj[k] = AM ? rdlane(wt, j + k) : 1;
                                dy[k].x = Td0[(size_t)yk * kWave + lane];
                                if (has1) dy[k].y = Td1[(size_t)yk * kWave + lane];
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        const bool t0 = r0 && dy[k].x != kInf && dy[k].x == dx.x + wj[k];
                        const bool t1 = r1 && dy[k].y != kInf && dy[k].y == dx.y + wj[k];
                        c0 += t0;
                        c1 += t1;
                        const uint64_t b0 = ballot(t0), b1 = ballot(t1);
                        if (lane == j + k) {
                            m0 = b0;
                            m1 = b1;
                        }
                    }
                }
                if (my < eb) {
                    Dg0[my] = m0;
                    if (has1) Dg1[my] = m1;
                }
            }
        } else {
            // no lane of either group reaches x: none of its arcs is on a shortest path
            for (int64_t e = ea + lane; e < eb; e += kWave) {
                Dg0[e] = 0ull;
                if (has1) Dg1[e] = 0ull;
            }
        }
        if (hub >= 0) {
            a.pd[((size_t)cg0 * a.nslots + part) * kWave + lane] = c0;
            if (has1) a.pd[((size_t)(cg0 + 1) * a.nslots + part) * kWave + lane] = c1;
        } else {
            const uint64_t b0 = count_finalize(a, (size_t)cg0 * n, cg0, x, dx.x, c0, lane);
            produced += __popcll(b0);
            if (CM) any0 |= b0;
            if (b0) act0 |= 1ull << (x - v0);
            if (has1) {
                const uint64_t b1 = count_finalize(a, (size_t)(cg0 + 1) * n, cg0 + 1, x, dx.y, c1, lane);
                produced += __popcll(b1);
                if (CM) any1 |= b1;
                if (b1) act1 |= 1ull << (x - v0);
            }
        }
    }
    if (hub < 0 && lane == 0) {
        if (a.nwide) {
            if (act0 | act1) or_run_bits(a.abits_n + (size_t)q * a.nwords, v0, act0 | act1);
        } else {
            if (act0) or_run_bits(a.abits_n + (size_t)cg0 * a.nwords, v0, act0);
            if (act1) or_run_bits(a.abits_n + (size_t)(cg0 + 1) * a.nwords, v0, act1);
        }
    }
    if (CM) {
        flush_colmask(a.colmask, a.ncg_all, cg0, any0);
        if (has1) flush_colmask(a.colmask, a.ncg_all, cg0 + 1, any1);
    }
}

// Finish (s, x) after a backward product contributed `acc` from `got`
// frontier successors.  Returns the lane mask of new frontier entries.
__device__ __forceinline__ uint64_t bwd_finalize(const BwdArgs &a, size_t cgv, int cg, int x,
                                                 int cx, double acc, int got, int lane,
                                                 unsigned long long &outs) {
    uint64_t bits = 0;
    const uint64_t gm = ballot(got > 0);
    if (lane == 0) outs += __popcll(gm);
    if (gm) {
        const size_t idx = (cgv + (size_t)x) * kWave + lane;
        bool done = false, front = false;
        double dep = 0.0;
        if (got > 0) {
            const int c = cx - got;
            const double z = a.zeta[idx] + acc;
            a.zeta[idx] = z;
            if (c == 0) {
                const double sg = a.tsig[idx];
                a.q[idx] = z + 1.0 / sg;
                a.cnt[idx] = -1;
                if (a.step) a.step[idx] = a.k;
                done = true;
                const bool self = a.src[cg * kWave + lane] == x;
                front = !self;
                if (!self) dep = z * sg;
            } else {
                a.cnt[idx] = c;
            }
        }
        bits = ballot(front);
        if (ballot(done)) {
            const double t = wave_sum(dep);
            if (lane == 0 && t != 0.0 && a.lam) a.lam[cgv + (size_t)x] += t;
        }
    }
    if (lane == 0) a.fbits_n[fb_index(a, cg, x)] = bits;
    return bits;
}

// ===================================================================== backward product
//
// MFBr's backward product as an instance of the generic pull product: for
// an owner x and its out-arcs x -> y, the action of an arc on the frontier
// entry of y is masked per lane by the stored shortest-path DAG -- the arc
// counts in lane s iff y is in the frontier of s and the arc is on a
// shortest path from s, the AND of two lane masks (the arc's tag) -- and
// (+) sums the frontier values q(s, y) of the counted arcs with their number.
// No distance is read, every counted arc belongs to a pending owner, and q is
// gathered only for counted lanes.  Every row of a run is visited: rows that
// count nothing clear their frontier lane masks.  W = 1: one column group;
// W = 2: a pair of groups (paired layout: lane masks [q][n][2], one activity
// bitmap per pair, one pass over the arcs and one 16-byte mask gather for
// both); a padding group (odd group count) has no state and counts nothing.
// CM: the served form records the columns that produced entries.
template <int AM_, int W, bool CM = false, int U_ = (W == 1 ? 4 : 2)>
struct BwdPull : PullDefaults {
    static constexpr int AM = AM_;
    static constexpr int U = U_;
    static constexpr int H = 4;
    static constexpr bool kEveryRow = true;
    struct Tag {
        uint64_t live[W];      // lanes for which the arc counts, per group
    };
    struct Row {
        double q[W];           // 0 where the arc does not count (a frontier value is > 0)
    };
    struct Acc {
        double z[W];
        int got[W];
    };
    struct Own {
        int cx[W];
    };
    const BwdArgs &a;
    const int q, lane, cg0;
    const bool has1;
    const size_t n;
    const uint32_t *bits;
    uint32_t *bits_n;
    unsigned long long &produced, &outs;
    uint64_t colany[W];

    __device__ __forceinline__ BwdPull(const BwdArgs &a_, int q_, unsigned long long &pr,
                                       unsigned long long &ou)
        : a(a_), q(q_), lane(threadIdx.x & (kWave - 1)), cg0(W * q_),
          has1(W == 2 && W * q_ + 1 < a_.ncg_all), n((size_t)a_.n),
          bits(a_.abits + (size_t)q_ * a_.nwords), bits_n(a_.abits_n + (size_t)q_ * a_.nwords),
          produced(pr), outs(ou) {
#pragma unroll
        for (int c = 0; c < W; c++) colany[c] = 0;
    }
    __device__ __forceinline__ bool in(int c) const { return c == 0 || has1; }
    __device__ __forceinline__ size_t cgv(int c) const { return (size_t)(cg0 + c) * n; }
    __device__ __forceinline__ Tag tag(int y, int64_t e) const {
        Tag t;
        if constexpr (W == 1) {
            t.live[0] = a.fbits[cgv(0) + (size_t)y] & a.dag[(size_t)cg0 * a.narcs + (size_t)e];
        } else {
            const ulonglong2 f = ((const ulonglong2 *)a.fbits)[(size_t)q * n + (size_t)y];
            const uint64_t *Dg = a.dag + (size_t)cg0 * a.narcs + (size_t)e;
            t.live[0] = f.x & Dg[0];
            t.live[1] = has1 ? f.y & Dg[a.narcs] : 0ull;
        }
        return t;
    }
    __device__ __forceinline__ bool live(const Tag &t) const {
        uint64_t any = 0;
#pragma unroll
        for (int c = 0; c < W; c++) any |= t.live[c];
        return any != 0;
    }
    __device__ __forceinline__ Row absent() const {
        Row r;
#pragma unroll
        for (int c = 0; c < W; c++) r.q[c] = 0.0;
        return r;
    }
    __device__ __forceinline__ Own none() const {
        Own o;
#pragma unroll
        for (int c = 0; c < W; c++) o.cx[c] = -1;
        return o;
    }
    __device__ __forceinline__ Row gather(int y, const Tag &t, int j) const {
        Row r = absent();
#pragma unroll
        for (int c = 0; c < W; c++) {
            if ((rdlane64(t.live[c], j) >> lane) & 1ull) r.q[c] = a.q[(cgv(c) + (size_t)y) * kWave + lane];
        }
        return r;
    }
    __device__ __forceinline__ Own own(int v0, int o) const {
        Own t;
#pragma unroll
        for (int c = 0; c < W; c++)
            t.cx[c] = in(c) ? a.cnt[(cgv(c) + (size_t)v0 + (size_t)o) * kWave + lane] : -1;
        return t;
    }
    __device__ __forceinline__ void batch(Row (&)[U], const int (&)[U]) const {}
    __device__ __forceinline__ void reset(Acc &x) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            x.z[c] = 0.0;
            x.got[c] = 0;
        }
    }
    __device__ __forceinline__ void fold(Acc &x, const Row &r, int, int) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            x.z[c] += r.q[c];
            x.got[c] += r.q[c] != 0.0;
        }
    }
    // element c of a W-array without indexing it by a runtime value (which
    // would put the array in scratch memory)
    template <typename T>
    __device__ __forceinline__ static T at(const T (&v)[W], int c) {
        return (W == 1 || c == 0) ? v[0] : v[W - 1];
    }
    __device__ __forceinline__ uint64_t finish(int v, const Acc &x, const Own &o) {
        if constexpr (W == 1) {
            const uint64_t b = bwd_finalize(a, cgv(0), cg0, v, o.cx[0], x.z[0], x.got[0], lane, outs);
            produced += __popcll(b);
            colany[0] |= b;
            return b;
        }
        uint64_t bb = 0;
        // one copy of the finish code for both groups (registers)
#pragma unroll 1
        for (int c = 0; c < W; c++) {
            if (!in(c)) break;
            const uint64_t b = bwd_finalize(a, cgv(c), cg0 + c, v, at(o.cx, c), at(x.z, c), at(x.got, c),
                                            lane, outs);
            produced += __popcll(b);
            bb |= b;
            if (W == 1 || c == 0) colany[0] |= b;
            else colany[W - 1] |= b;
        }
        return bb;
    }
    __device__ __forceinline__ void idle(int v) const {
        if constexpr (W == 1) {
            if (lane == 0) a.fbits_n[cgv(0) + (size_t)v] = 0ull;
        } else {
            if (lane < 2) a.fbits_n[((size_t)q * n + (size_t)v) * 2 + lane] = 0ull;
        }
    }
    __device__ __forceinline__ size_t slot(int c, int part) const {
        return ((size_t)(cg0 + c) * a.nslots + part) * kWave + lane;
    }
    __device__ __forceinline__ void store(int part, const Acc &x) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            a.pd[slot(c, part)] = x.got[c];
            a.pm[slot(c, part)] = x.z[c];
        }
    }
    __device__ __forceinline__ Acc load(int part) const {
        Acc x;
        reset(x);
#pragma unroll
        for (int c = 0; c < W; c++) {
            if (!in(c)) continue;
            x.got[c] = a.pd[slot(c, part)];
            x.z[c] = a.pm[slot(c, part)];
        }
        return x;
    }
    // slice partials summed in slice order
    __device__ __forceinline__ void merge(Acc &x, const Acc &y) const {
#pragma unroll
        for (int c = 0; c < W; c++) {
            x.z[c] += y.z[c];
            x.got[c] += y.got[c];
        }
    }
    __device__ __forceinline__ uint64_t finish_hub(int v, const Acc &x) {
        return finish(v, x, own(v, 0));
    }
    // record, per group, the columns that produced entries (served form)
    __device__ __forceinline__ void flush() const {
#pragma unroll
        for (int c = 0; c < W; c++)
            if (in(c) && (W == 1 || CM)) flush_colmask(a.colmask, a.ncg_all, cg0 + c, colany[c]);
    }
};

// One pull task of a backward product for column group cg.
template <int AM>
__device__ __forceinline__ void bwd_task(const BwdArgs &a, int cg, int t, unsigned long long &produced,
                                         unsigned long long &outs) {
    BwdPull<AM, 1> p(a, cg, produced, outs);
    pull_task_owner(p, a.tasks + t, a.rp, a.arcs);
    p.flush();
}

__device__ __forceinline__ void bwd_hub(const BwdArgs &a, int cg, int h, unsigned long long &produced,
                                        unsigned long long &outs) {
    BwdPull<0, 1> p(a, cg, produced, outs);
    pull_hub(p, a.hubs + h);
    p.flush();
}

// The same for the pair of column groups q (paired layout).
template <int AM, bool CM>
__device__ __forceinline__ void bwd_task_w(const BwdArgs &a, int q, int t, unsigned long long &produced,
                                           unsigned long long &outs) {
    BwdPull<AM, 2, CM> p(a, q, produced, outs);
    pull_task_owner(p, a.tasks + t, a.rp, a.arcs);
    p.flush();
}

__device__ __forceinline__ void bwd_hub_w(const BwdArgs &a, int q, int h, unsigned long long &produced,
                                          unsigned long long &outs) {
    BwdPull<0, 2, true> p(a, q, produced, outs);
    pull_hub(p, a.hubs + h);
    p.flush();
}


// ===================================================================== grid kernels
// The pull kernels are latency bound, so waves in flight matter most.  A SIMD
// holds 800 scalar registers, handed out in granules, so eight waves per SIMD
// fit only when a wave takes at most 96 of them in all (VCC included); the
// budget below (which yields that total) makes the compiler keep to it,
// spilling the odd uniform value to a vector lane, where it would otherwise
// use a few more and silently drop to seven waves.
#define MFBC_PULL_SGPRS __attribute__((amdgpu_num_sgpr(98)))

// L: the launch covers the ncg column groups listed in a.cglist (served form)
// rather than groups 0..ncg-1; a separate instantiation keeps the plain path's
// code free of the list.
template <bool L>
__device__ __forceinline__ int pick_cg(const int32_t *cglist, int cg) {
    if constexpr (L) return cglist[cg];
    return cg;
}

template <int AM, bool L>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_fwd_pull(FwdArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;                       // column-group major
    unsigned long long produced = 0, outs = 0;
    if (cg < a.ncg) fwd_task<AM>(a, pick_cg<L>(a.cglist, cg), wid - cg * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

// A merge whose product was skipped (see live_prev) only clears the next
// product's counters: no hub partial was written and the frontier it would
// clear is empty.
template <bool L>
__global__ __launch_bounds__(kBlock) void k_fwd_merge(FwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.ncg_all, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) fwd_hub(a, pick_cg<L>(a.cglist, cg), wid - cg * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

// Wide forward product: wave = (wide group, task), group-major.  With L the
// launch covers the a.nwide wide groups listed in a.cglist (served form),
// else groups 0 .. a.nwide-1; the merge clears a.nwide_all bitmap planes.
template <int AM, int W, bool L>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_fwd_pull_w(FwdArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int q = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (q < a.nwide) fwd_task_w<AM, W>(a, pick_cg<L>(a.cglist, q), wid - q * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

template <int W, bool L>
__global__ __launch_bounds__(kBlock) void k_fwd_merge_w(FwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.nwide_all, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int q = a.nhubs ? wid / a.nhubs : a.nwide;
    if (q < a.nwide) fwd_hub_w<W>(a, pick_cg<L>(a.cglist, q), wid - q * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

template <int AM, bool L>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_bwd_count(BwdArgs a) {
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;                       // column-group major
    unsigned long long produced = 0;
    if (cg < a.ncg) count_task<AM>(a, pick_cg<L>(a.cglist, cg), wid - cg * a.ntasks, produced);
    flush_counts(produced, 0, 0, 0, a.ctr);
}

// Paired counting product: wave = (pair, task).  Plain path: every pair of
// the batch; with L, the a.nwide pairs listed in a.cglist (served form).
// Both FULL variants are launched: the one that does not match the flag of
// the compact tau copy (a.tau_full, written by the pass that made the copy)
// returns at once, so each variant keeps its own register allocation.
template <int AM, bool L, bool FULL>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS __attribute__((amdgpu_waves_per_eu(7))) void k_bwd_count_w(BwdArgs a) {
    if ((uni(*a.tau_full) != 0) != FULL) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int q = wid / a.ntasks;
    const int np = L ? a.nwide : (a.ncg + 1) / 2;
    unsigned long long produced = 0;
    if (q < np) count_task_w<AM, L, FULL>(a, pick_cg<L>(a.cglist, q), wid - q * a.ntasks, produced);
    flush_counts(produced, 0, 0, 0, a.ctr);
}

template <bool L>
__global__ __launch_bounds__(kBlock) void k_bwd_count_merge(BwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) count_hub(a, pick_cg<L>(a.cglist, cg), wid - cg * a.nhubs, produced);
    flush_counts(produced, 0, 0, 0, a.ctr);
}

template <int AM, bool L>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS __attribute__((amdgpu_waves_per_eu(8))) void k_bwd_pull(BwdArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;                       // column-group major
    unsigned long long produced = 0, outs = 0;
    if (cg < a.ncg) bwd_task<AM>(a, pick_cg<L>(a.cglist, cg), wid - cg * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

// Paired backward product: wave = (pair, task), pair-major; with L over the
// a.nwide pairs listed in a.cglist (served form).
template <int AM, bool L>
__global__ __launch_bounds__(kBlock) MFBC_PULL_SGPRS void k_bwd_pull_w(BwdArgs a) {
    if (!live_prev(a.prev_ctr)) return;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int q = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (q < a.nwide) bwd_task_w<AM, L>(a, pick_cg<L>(a.cglist, q), wid - q * a.ntasks, produced, outs);
    flush_counts(produced, outs, 0, 0, a.ctr);
}

template <bool L>
__global__ __launch_bounds__(kBlock) void k_bwd_merge_w(BwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.nwide_all, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int q = a.nhubs ? wid / a.nhubs : a.nwide;
    if (q < a.nwide) bwd_hub_w(a, pick_cg<L>(a.cglist, q), wid - q * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

template <bool L>
__global__ __launch_bounds__(kBlock) void k_bwd_merge(BwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (!live_prev(a.prev_ctr)) {
        if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
        return;
    }
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.ncg_all, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) bwd_hub(a, pick_cg<L>(a.cglist, cg), wid - cg * a.nhubs, produced, outs);
    flush_counts(produced, outs, nv, na, a.ctr);
}

}  // namespace
}  // namespace mfbc
