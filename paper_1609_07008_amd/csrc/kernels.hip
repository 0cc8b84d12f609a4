// HIP kernels of libmfbc for gfx950 (CDNA4, wave64).
//
// Both products of the method are computed in *pull* form: the wave that
// owns output row (v, column group cg) walks v's adjacency row once and
// combines, lane by lane (one lane per source column), the frontier tuples of
// the neighbours that are active.  Every output entry has exactly one owner
// per product, so no atomics touch the tuples and results are deterministic
// (fixed CSR order inside a row, fixed slice order when a hub row is split).
//
//  * Forward product (Section 4.1, Algorithm 1):  G = F (+,f) A  with the
//    multpath monoid (least weight, multiplicities of ties added) and
//    f(a, w) = (a.w + w, a.m); then T := T (+) G and the next frontier keeps
//    the entries of G that are not heavier than T.
//  * Counting product (Algorithm 2, initialisation): for each reachable
//    (s, x), the number of successors y with tau(s,x) + A(x,y) = tau(s,y).
//    Under the centpath monoid (greatest weight wins, ties add) applied to
//    g(a, w) = (a.w - w, ...) only successors reach weight tau(s,x); all other
//    neighbours are lighter, so the product reduces to this equality test.
//  * Backward product (Algorithm 2, loop): for each pending (s, x), the sum of
//    the frontier values q(s,y) = zeta(s,y) + 1/sigma(s,y) over frontier
//    successors y, and the number of them, which is taken off x's counter;
//    x joins the next frontier when its counter reaches zero.
//  * lambda (Algorithm 3): delta(s,x) = zeta(s,x) * sigma(s,x) is added to a
//    per-(column group, vertex) partial when (s,x) completes; the source's
//    own entry is excluded (sigma(s,t,s) = 0 in Section 2.4).
//
// Activity filter: a one-bit-per-vertex bitmap (any column active) is
// checked per arc first (n/8 bytes, resident in L2), then the 64-bit lane
// mask of (u, cg); only lanes whose bit is set load the frontier tuple.
#include "mfbc_internal.h"

namespace mfbc {
namespace {

__device__ __forceinline__ int rdlane(int x, int j) { return __builtin_amdgcn_readlane(x, j); }

__device__ __forceinline__ uint64_t rdlane64(uint64_t x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ int64_t uni64(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Set the bits of `mask` (bit i = vertex v0 + i) in a vertex bitmap.
__device__ __forceinline__ void or_run_bits(uint32_t *bm, int v0, uint64_t mask) {
    const int w0 = v0 >> 5, sh = v0 & 31;
    const uint64_t lo = mask << sh;
    const uint32_t hi = sh ? (uint32_t)(mask >> (64 - sh)) : 0u;
    if ((uint32_t)lo) atomicOr(bm + w0, (uint32_t)lo);
    if ((uint32_t)(lo >> 32)) atomicOr(bm + w0 + 1, (uint32_t)(lo >> 32));
    if (hi) atomicOr(bm + w0 + 2, hi);
}

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
            while (w) {
                const int b = __ffs(w) - 1;
                w &= w - 1;
                const int u = i * 32 + b;
                na += (unsigned long long)(rp[u + 1] - rp[u]);
            }
        }
    }
}

// Arcs of the current 64-arc chunk that belong to the owner whose row ends
// at `vend` (chunk starts at arc e).
__device__ __forceinline__ uint64_t owner_mask(int64_t e, int64_t vend) {
    const int64_t k = vend - e;
    return k >= 64 ? ~0ull : ((1ull << k) - 1ull);
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

// Arc access: AM = 0 unweighted (col), 1 packed (col | w << cb), 2 separate arrays.
struct ArcSrc {
    const int32_t *col;
    const int32_t *w;
    const uint32_t *pk;
    int cb;
    uint32_t cmask;
};

template <int AM>
__device__ __forceinline__ void load_arc(const ArcSrc &s, int64_t e, int &u, int &wt) {
    if (AM == 1) {
        const uint32_t p = s.pk[e];
        u = (int)(p & s.cmask);
        wt = (int)(p >> s.cb);
    } else {
        u = s.col[e];
        wt = AM == 2 ? s.w[e] : 1;
    }
}

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
    int32_t *flags;
    uint64_t *fmask;           // trace (nullable)
    uint32_t *clear_bits;      // merge: bitmaps to clear (F_{j-1}'s), ncg planes
    unsigned long long *clear_ctr;  // merge: counter slots of product j+1
};

// T := T (+) G at (v, cg); writes the next frontier row.  Returns the lane
// mask of the frontier entries produced.
__device__ __forceinline__ uint64_t fwd_finalize(const FwdArgs &a, size_t cgv, int v, int bd,
                                                 double bm, int lane, unsigned long long &outs) {
    const bool has = bd != kInf;
    uint64_t bits = 0;
    const uint64_t hm = ballot(has);
    outs += __popcll(hm);
    if (hm) {
        const size_t idx = (cgv + (size_t)v) * kWave + lane;
        bool keep = false;
        if (has) {
            const int td = a.tdist[idx];
            if (bd < td) {
                a.tdist[idx] = bd;
                a.tsig[idx] = bm;
                keep = true;
                if (__builtin_isinf(bm)) a.flags[0] = 1;
            } else if (bd == td) {
                const double s = a.tsig[idx] + bm;
                a.tsig[idx] = s;
                keep = true;
                if (__builtin_isinf(s)) a.flags[0] = 1;
            }
        }
        bits = ballot(keep);
        if (bits) {
            uint32_t t = kSent;
            if (keep) {
                const double mmax = (double)((1u << a.mb) - 1u);
                const uint32_t ms = bm <= mmax ? (uint32_t)bm : 0u;
                if (ms == 0u) a.fsig_n[idx] = bm;
                t = ((uint32_t)bd << a.mb) | ms;
                if (a.fmask && a.j <= 64) a.fmask[idx] |= 1ull << (a.j - 1);
            }
            a.ftup_n[idx] = t;
        }
    }
    return bits;
}

constexpr int kFwdUnroll = 8;

template <int AM>
__global__ __launch_bounds__(kBlock) void k_fwd_pull(FwdArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;                       // column-group major
    unsigned long long produced = 0, outs = 0;
    if (cg < a.ncg) {
        const Task *tp = a.tasks + (wid - cg * a.ntasks);
        const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
        const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        const uint32_t *Ft = a.ftup + cgv * kWave;
        const double *Fm = a.fsig + cgv * kWave;
        const uint32_t *Ab = a.abits + (size_t)cg * a.nwords;
        const uint32_t mmask = (1u << a.mb) - 1u;
        int v = v0;
        int64_t vend = hub >= 0 ? e1 : a.rp[v0 + 1];
        int bd = kInf;
        double bm = 0.0;
        uint64_t run_act = 0;
        for (int64_t e = e0; e < e1; e += kWave) {
            const int64_t my = e + lane;
            int u = 0, wt = 1;
            bool act = false;
            if (my < e1) {
                load_arc<AM>(a.arcs, my, u, wt);
                act = (Ab[u >> 5] >> (u & 31)) & 1u;
            }
            uint64_t am = ballot(act);
            while (am) {
                const int j0 = __ffsll((unsigned long long)am) - 1;
                if (hub < 0) {
                    while (e + j0 >= vend) {
                        const uint64_t b = fwd_finalize(a, cgv, v, bd, bm, lane, outs);
                        produced += __popcll(b);
                        if (b) run_act |= 1ull << (v - v0);
                        ++v;
                        vend = a.rp[v + 1];
                        bd = kInf;
                        bm = 0.0;
                    }
                }
                // up to kFwdUnroll active arcs of the same owner, loads issued together
                uint64_t cand = am & owner_mask(e, vend);
                int js[kFwdUnroll];
#pragma unroll
                for (int k = 0; k < kFwdUnroll; k++) {
                    js[k] = cand ? __ffsll((unsigned long long)cand) - 1 : -1;
                    cand &= cand - 1;
                }
                uint32_t tk[kFwdUnroll];
                int uk[kFwdUnroll], wk[kFwdUnroll];
#pragma unroll
                for (int k = 0; k < kFwdUnroll; k++) {
                    tk[k] = kSent;
                    uk[k] = 0;
                    wk[k] = 0;
                    if (js[k] >= 0) {
                        am &= ~(1ull << js[k]);
                        uk[k] = rdlane(u, js[k]);
                        wk[k] = AM ? rdlane(wt, js[k]) : 1;
                        tk[k] = Ft[(size_t)uk[k] * kWave + lane];
                    }
                }
                double mk[kFwdUnroll];
#pragma unroll
                for (int k = 0; k < kFwdUnroll; k++) {
                    mk[k] = 0.0;
                    if (tk[k] != kSent) {
                        const uint32_t ms = tk[k] & mmask;
                        mk[k] = ms ? (double)ms : Fm[(size_t)uk[k] * kWave + lane];
                    }
                }
#pragma unroll
                for (int k = 0; k < kFwdUnroll; k++) {
                    if (tk[k] != kSent) {
                        const int d = (int)(tk[k] >> a.mb) + wk[k];
                        if (d < bd) {
                            bd = d;
                            bm = mk[k];
                        } else if (d == bd) {
                            bm += mk[k];
                        }
                    }
                }
            }
        }
        if (hub < 0) {
            while (v < v1) {
                const uint64_t b = fwd_finalize(a, cgv, v, bd, bm, lane, outs);
                produced += __popcll(b);
                if (b) run_act |= 1ull << (v - v0);
                ++v;
                bd = kInf;
                bm = 0.0;
            }
            if (lane == 0 && run_act) or_run_bits(a.abits_n + (size_t)cg * a.nwords, v0, run_act);
        } else {
            const size_t pidx = ((size_t)cg * a.nslots + part) * kWave + lane;
            a.pd[pidx] = bd;
            a.pm[pidx] = bm;
        }
    }
    flush_counts(produced, outs, 0, 0, a.ctr);
}

// Combine the slices of split rows (fixed slice order) and finish them;
// also clears the previous frontier's bitmaps (counting the vertices active
// in some column and their arcs) and the next product's counters.
__global__ __launch_bounds__(kBlock) void k_fwd_merge(FwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.ncg, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) {
        const Hub *hp = a.hubs + (wid - cg * a.nhubs);
        const int v = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        int bd = kInf;
        double bm = 0.0;
        for (int p = first; p < first + np; p++) {
            const size_t pidx = ((size_t)cg * a.nslots + p) * kWave + lane;
            const int d = a.pd[pidx];
            const double m = a.pm[pidx];
            if (d < bd) {
                bd = d;
                bm = m;
            } else if (d == bd && d != kInf) {
                bm += m;
            }
        }
        const uint64_t b = fwd_finalize(a, cgv, v, bd, bm, lane, outs);
        produced += __popcll(b);
        if (b && lane == 0) atomicOr(a.abits_n + (size_t)cg * a.nwords + (v >> 5), 1u << (v & 31));
    }
    flush_counts(produced, outs, nv, na, a.ctr);
}

// ===================================================================== backward
struct BwdArgs {
    const Task *tasks;
    const Hub *hubs;
    int ntasks, nhubs, nslots, ncg, n, k, nwords;
    const int64_t *rp;         // out-arcs
    const int32_t *col;
    const int32_t *w;
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
    uint32_t *clear_bits;      // ncg planes
    unsigned long long *clear_ctr;
};

// Per-vertex finish of the counting product: counters, leaves, zeta = 0.
__device__ __forceinline__ uint64_t count_finalize(const BwdArgs &a, size_t cgv, int cg, int x,
                                                   int dx, int c, int lane) {
    const size_t idx = (cgv + (size_t)x) * kWave + lane;
    const bool reach = dx != kInf;
    const bool leaf = reach && c == 0;
    const bool front = leaf && a.src[cg * kWave + lane] != x;
    a.cnt[idx] = (reach && c > 0) ? c : -1;
    a.zeta[idx] = 0.0;
    a.step[idx] = leaf ? 0 : -1;
    if (leaf) a.q[idx] = 1.0 / a.tsig[idx];
    const uint64_t bits = ballot(front);
    if (lane == 0) a.fbits_n[cgv + (size_t)x] = bits;
    return bits;
}

// Counting product: every arc x -> y, lane test tau(y) == tau(x) + w.
template <bool W>
__global__ __launch_bounds__(kBlock) void k_bwd_count(BwdArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;
    unsigned long long produced = 0;
    if (cg < a.ncg) {
        const Task *tp = a.tasks + (wid - cg * a.ntasks);
        const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
        const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        const int32_t *Td = a.tdist + cgv * kWave;
        uint64_t run_act = 0;
        const int xa = v0, xb = hub >= 0 ? v0 + 1 : v1;
        for (int x = xa; x < xb; x++) {
            const int dx = Td[(size_t)x * kWave + lane];
            const bool reach = dx != kInf;
            const int64_t ea = hub >= 0 ? e0 : a.rp[x];
            const int64_t eb = hub >= 0 ? e1 : a.rp[x + 1];
            int c = 0;
            if (ballot(reach)) {
                for (int64_t e = ea; e < eb; e += kWave) {
                    const int64_t my = e + lane;
                    int y = 0, wt = 1;
                    if (my < eb) {
                        y = a.col[my];
                        if (W) wt = a.w[my];
                    }
                    const int cnt = (int)((eb - e) < kWave ? (eb - e) : kWave);
                    for (int j = 0; j < cnt; j += 8) {
                        int dy[8], wj[8];
#pragma unroll
                        for (int k = 0; k < 8; k++) {
                            dy[k] = kInf;
                            wj[k] = 0;
                            if (j + k < cnt) {
                                const int yk = rdlane(y, j + k);
                                wj[k] = W ? rdlane(wt, j + k) : 1;
                                if (reach) dy[k] = Td[(size_t)yk * kWave + lane];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 8; k++)
                            if (reach && dy[k] != kInf && dy[k] == dx + wj[k]) c++;
                    }
                }
            }
            if (hub >= 0) {
                a.pd[((size_t)cg * a.nslots + part) * kWave + lane] = c;
            } else {
                const uint64_t b = count_finalize(a, cgv, cg, x, dx, c, lane);
                produced += __popcll(b);
                if (b) run_act |= 1ull << (x - v0);
            }
        }
        if (hub < 0 && lane == 0 && run_act)
            or_run_bits(a.abits_n + (size_t)cg * a.nwords, v0, run_act);
    }
    flush_counts(produced, 0, 0, 0, a.ctr);
}

__global__ __launch_bounds__(kBlock) void k_bwd_count_merge(BwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) {
        const Hub *hp = a.hubs + (wid - cg * a.nhubs);
        const int x = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        int c = 0;
        for (int p = first; p < first + np; p++) c += a.pd[((size_t)cg * a.nslots + p) * kWave + lane];
        const int dx = a.tdist[(cgv + (size_t)x) * kWave + lane];
        const uint64_t b = count_finalize(a, cgv, cg, x, dx, c, lane);
        produced += __popcll(b);
        if (b && lane == 0) atomicOr(a.abits_n + (size_t)cg * a.nwords + (x >> 5), 1u << (x & 31));
    }
    flush_counts(produced, 0, 0, 0, a.ctr);
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
                a.step[idx] = a.k;
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
            if (lane == 0 && t != 0.0) a.lam[cgv + (size_t)x] += t;
        }
    }
    if (lane == 0) a.fbits_n[cgv + (size_t)x] = bits;
    return bits;
}

template <bool W>
__global__ __launch_bounds__(kBlock) void k_bwd_pull(BwdArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int cg = wid / a.ntasks;
    unsigned long long produced = 0, outs = 0;
    if (cg < a.ncg) {
        const Task *tp = a.tasks + (wid - cg * a.ntasks);
        const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
        const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        const int32_t *Td = a.tdist + cgv * kWave;
        const double *Q = a.q + cgv * kWave;
        const uint64_t *Fb = a.fbits + cgv;
        const uint32_t *Ab = a.abits + (size_t)cg * a.nwords;
        int x = v0;
        int64_t vend = hub >= 0 ? e1 : a.rp[v0 + 1];
        bool loaded = false;
        int cx = -1, dx = kInf, got = 0;
        double acc = 0.0;
        uint64_t run_act = 0;
        for (int64_t e = e0; e < e1; e += kWave) {
            const int64_t my = e + lane;
            int y = 0, wt = 1;
            uint64_t fb = 0;
            if (my < e1) {
                y = a.col[my];
                if (W) wt = a.w[my];
                if ((Ab[y >> 5] >> (y & 31)) & 1u) fb = Fb[y];
            }
            uint64_t am = ballot(fb != 0);
            while (am) {
                const int j0 = __ffsll((unsigned long long)am) - 1;
                if (hub < 0) {
                    while (e + j0 >= vend) {
                        if (loaded) {
                            const uint64_t b = bwd_finalize(a, cgv, cg, x, cx, acc, got, lane, outs);
                            produced += __popcll(b);
                            if (b) run_act |= 1ull << (x - v0);
                        } else if (lane == 0) {
                            a.fbits_n[cgv + (size_t)x] = 0ull;
                        }
                        ++x;
                        vend = a.rp[x + 1];
                        loaded = false;
                        got = 0;
                        acc = 0.0;
                    }
                }
                if (!loaded) {
                    const size_t idx = (cgv + (size_t)x) * kWave + lane;
                    cx = a.cnt[idx];
                    dx = Td[(size_t)x * kWave + lane];
                    loaded = true;
                }
                const bool pend = cx > 0;
                uint64_t cand = am & owner_mask(e, vend);
                if (!ballot(pend)) {
                    am &= ~cand;            // nothing of x is pending: skip its arcs here
                    continue;
                }
                int js[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    js[k] = cand ? __ffsll((unsigned long long)cand) - 1 : -1;
                    cand &= cand - 1;
                }
                // distances first; the frontier value q is loaded only for
                // lanes whose arc is a shortest-path arc (few per row)
                int dy[4], wk[4], yk[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    dy[k] = kInf;
                    wk[k] = 0;
                    yk[k] = 0;
                    if (js[k] >= 0) {
                        am &= ~(1ull << js[k]);
                        yk[k] = rdlane(y, js[k]);
                        wk[k] = W ? rdlane(wt, js[k]) : 1;
                        const uint64_t fbj = rdlane64(fb, js[k]);
                        if (pend && ((fbj >> lane) & 1ull)) dy[k] = Td[(size_t)yk[k] * kWave + lane];
                    }
                }
                double qy[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const bool tight = dy[k] != kInf && dy[k] == dx + wk[k];
                    qy[k] = tight ? Q[(size_t)yk[k] * kWave + lane] : 0.0;
                    if (tight) got++;
                }
#pragma unroll
                for (int k = 0; k < 4; k++) acc += qy[k];
            }
        }
        if (hub < 0) {
            while (x < v1) {
                if (loaded) {
                    const uint64_t b = bwd_finalize(a, cgv, cg, x, cx, acc, got, lane, outs);
                    produced += __popcll(b);
                    if (b) run_act |= 1ull << (x - v0);
                } else if (lane == 0) {
                    a.fbits_n[cgv + (size_t)x] = 0ull;
                }
                ++x;
                loaded = false;
                got = 0;
                acc = 0.0;
            }
            if (lane == 0 && run_act) or_run_bits(a.abits_n + (size_t)cg * a.nwords, v0, run_act);
        } else {
            const size_t pidx = ((size_t)cg * a.nslots + part) * kWave + lane;
            a.pd[pidx] = got;
            a.pm[pidx] = acc;
        }
    }
    flush_counts(produced, outs, 0, 0, a.ctr);
}

__global__ __launch_bounds__(kBlock) void k_bwd_merge(BwdArgs a) {
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    unsigned long long nv = 0, na = 0;
    clear_and_count(a.clear_bits, a.nwords, a.ncg, a.rp, nv, na);
    if (gtid < 4 * kCounterSlots) a.clear_ctr[gtid] = 0ull;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    unsigned long long produced = 0, outs = 0;
    const int cg = a.nhubs ? wid / a.nhubs : a.ncg;
    if (cg < a.ncg) {
        const Hub *hp = a.hubs + (wid - cg * a.nhubs);
        const int x = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
        const size_t cgv = (size_t)cg * (size_t)a.n;
        int got = 0;
        double acc = 0.0;
        for (int p = first; p < first + np; p++) {
            const size_t pidx = ((size_t)cg * a.nslots + p) * kWave + lane;
            got += a.pd[pidx];
            acc += a.pm[pidx];
        }
        const int cx = a.cnt[(cgv + (size_t)x) * kWave + lane];
        const uint64_t b = bwd_finalize(a, cgv, cg, x, cx, acc, got, lane, outs);
        produced += __popcll(b);
        if (b && lane == 0) atomicOr(a.abits_n + (size_t)cg * a.nwords + (x >> 5), 1u << (x & 31));
    }
    flush_counts(produced, outs, nv, na, a.ctr);
}

// ===================================================================== setup / io
__global__ void k_set_sources(int32_t *src, int total, int nb, const int32_t *in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) src[i] = i < nb ? in[i] : -1;
}

// T = (INF, 0) everywhere, both frontier bitmaps cleared, counters zeroed.
__global__ void k_fwd_fill(int32_t *tdist, double *tsig, size_t total, uint32_t *ab0, uint32_t *ab1,
                           size_t nab, unsigned long long *ctr, int nctr, int32_t *flags,
                           uint64_t *fmask) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < total; i += stride) {
        tdist[i] = kInf;
        tsig[i] = 0.0;
        if (fmask) fmask[i] = 0ull;
    }
    for (size_t i = t0; i < nab; i += stride) {
        ab0[i] = 0u;
        ab1[i] = 0u;
    }
    if (t0 < (size_t)nctr) ctr[t0] = 0ull;
    if (t0 == 0) flags[0] = 0;
}

// Rows of the sources in the first frontier start with every lane absent.
__global__ void k_fwd_seed_rows(const int32_t *src, int nb, int n, uint32_t *ftup) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const size_t row = ((size_t)(c / kWave) * n + src[c]) * kWave;
    for (int l = 0; l < kWave; l++) ftup[row + l] = kSent;
}

// The sources themselves: T(s, s) = (0, 1) and the first frontier {s}
// carrying (0, 1).
__global__ void k_fwd_seed(const int32_t *src, int nb, int n, int nwords, int32_t *tdist,
                           double *tsig, uint32_t *ftup, uint32_t *abits) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int v = src[c];
    const int cg = c / kWave, lane = c % kWave;
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    tdist[idx] = 0;
    tsig[idx] = 1.0;
    ftup[idx] = 1u;                      // weight 0, multiplicity 1 inline
    atomicOr(abits + (size_t)cg * nwords + (v >> 5), 1u << (v & 31));
}

__global__ void k_zero_f64(double *p, size_t total) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) p[i] = 0.0;
}

__global__ void k_lambda_reduce(const double *lam, int ncg, int n, double *bc) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double t = 0.0;
    for (int cg = 0; cg < ncg; cg++) t += lam[(size_t)cg * n + v];
    bc[v] = t;
}

// Tile transposes between [cg][v][64] tiles and source-major rows [s][v],
// 64 x 64 per block through LDS (padded against bank conflicts).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tiles_to_rows(const T *tiles, T *rows, int n, int nb) {
    __shared__ T sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) sh[r][c] = tiles[((size_t)cg * n + v) * 64 + c];
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        if (s < nb && v < n) rows[(size_t)s * n + v] = sh[c][r];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rows_to_tiles(const T *rows, T *tiles, int n, int nb,
                                                          T pad) {
    __shared__ T sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        sh[c][r] = (s < nb && v < n) ? rows[(size_t)s * n + v] : pad;
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) tiles[((size_t)cg * n + v) * 64 + c] = sh[r][c];
    }
}

// delta(s, v) = zeta(s, v) * sigma(s, v), 0 at the source and where unreachable.
__global__ __launch_bounds__(kBlock) void k_delta_rows(const double *zeta, const double *tsig,
                                                       const int32_t *tdist, const int32_t *src,
                                                       double *rows, int n, int nb) {
    __shared__ double sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) {
            const size_t idx = ((size_t)cg * n + v) * 64 + c;
            const bool ok = tdist[idx] != kInf && src[cg * 64 + c] != v;
            sh[r][c] = ok ? zeta[idx] * tsig[idx] : 0.0;
        }
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        if (s < nb && v < n) rows[(size_t)s * n + v] = sh[c][r];
    }
}

inline int blocks_for(size_t work, int per_block, int cap = 1 << 20) {
    size_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

}  // namespace

// ===================================================================== launchers
static ArcSrc arc_src(const Csr &c) {
    ArcSrc r{};
    r.col = c.col;
    r.w = c.w;
    r.pk = c.pk;
    r.cb = c.cb;
    r.cmask = c.cb >= 32 ? 0xffffffffu : ((1u << c.cb) - 1u);
    return r;
}

static int arc_mode(const Csr &c) { return c.w == nullptr ? 0 : (c.pk ? 1 : 2); }

static FwdArgs fwd_args(mfbc_graph *g, int ncg, int j, bool trace) {
    Workspace &ws = g->ws;
    const int b = (j - 1) & 1;  // buffer holding F_{j-1}
    FwdArgs a{};
    a.tasks = g->plan_in.tasks;
    a.hubs = g->plan_in.hubs;
    a.ntasks = g->plan_in.ntasks;
    a.nhubs = g->plan_in.nhubs;
    a.nslots = g->plan_in.nslots;
    a.ncg = ncg;
    a.n = g->n;
    a.j = j;
    a.nwords = (g->n + 31) / 32;
    a.mb = g->mb;
    a.rp = g->in.rp;
    a.arcs = arc_src(g->in);
    a.abits = ws.abits[b];
    a.ftup = (const uint32_t *)ws.fdist[b];
    a.fsig = ws.fsig[b];
    a.tdist = ws.tdist;
    a.tsig = ws.tsig;
    a.abits_n = ws.abits[b ^ 1];
    a.ftup_n = (uint32_t *)ws.fdist[b ^ 1];
    a.fsig_n = ws.fsig[b ^ 1];
    a.pd = ws.pd;
    a.pm = ws.pm;
    a.ctr = ws.counters + (size_t)(j % kCounterRing) * 4 * kCounterSlots;
    a.flags = ws.flags;
    a.fmask = trace ? ws.fmask : nullptr;
    a.clear_bits = ws.abits[b];
    a.clear_ctr = ws.counters + (size_t)((j + 1) % kCounterRing) * 4 * kCounterSlots;
    return a;
}

void launch_set_sources(mfbc_graph *g, int ncg, int nb, const int32_t *d_sources, hipStream_t s) {
    const int total = ncg * kWave;
    hipLaunchKernelGGL(k_set_sources, dim3(blocks_for(total, 256)), dim3(256), 0, s, g->ws.src,
                       total, nb, d_sources);
}

void launch_fwd_init(mfbc_graph *g, int ncg, int nb, hipStream_t s) {
    Workspace &ws = g->ws;
    const size_t total = (size_t)ncg * g->n * kWave;
    const int nwords = (g->n + 31) / 32;
    hipLaunchKernelGGL(k_fwd_fill, dim3(blocks_for(total, 256, 65536)), dim3(256), 0, s, ws.tdist,
                       ws.tsig, total, ws.abits[0], ws.abits[1], (size_t)ncg * nwords,
                       ws.counters, kCounterRing * 4 * kCounterSlots, ws.flags,
                       ws.fmask && ws.fmask_ncg >= ncg ? ws.fmask : nullptr);
    hipLaunchKernelGGL(k_fwd_seed_rows, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src, nb,
                       g->n, (uint32_t *)ws.fdist[0]);
    hipLaunchKernelGGL(k_fwd_seed, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                       nwords, ws.tdist, ws.tsig, (uint32_t *)ws.fdist[0], ws.abits[0]);
}

void launch_fwd_product(mfbc_graph *g, int ncg, int j, bool trace, hipStream_t s,
                        hipEvent_t *ev) {
    FwdArgs a = fwd_args(g, ncg, j, trace);
    if (ev) hipEventRecord(ev[0], s);
    const size_t waves = (size_t)a.ntasks * ncg;
    const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
    switch (arc_mode(g->in)) {
        case 0: hipLaunchKernelGGL(k_fwd_pull<0>, dim3(grid), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_fwd_pull<1>, dim3(grid), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL(k_fwd_pull<2>, dim3(grid), dim3(kBlock), 0, s, a); break;
    }
    if (ev) hipEventRecord(ev[1], s);
    const size_t mw = (size_t)a.nhubs * ncg;
    int mgrid = blocks_for(mw, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_fwd_merge, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev) hipEventRecord(ev[2], s);
}

static BwdArgs bwd_args(mfbc_graph *g, int ncg, int k) {
    Workspace &ws = g->ws;
    // k = 0: counting product writes B_0 into buffer 0; product k reads
    // B_{k-1} from buffer (k-1)&1 and writes B_k into buffer k&1.
    const int bn = k & 1, b = bn ^ 1;
    BwdArgs a{};
    a.tasks = g->plan_out.tasks;
    a.hubs = g->plan_out.hubs;
    a.ntasks = g->plan_out.ntasks;
    a.nhubs = g->plan_out.nhubs;
    a.nslots = g->plan_out.nslots;
    a.ncg = ncg;
    a.n = g->n;
    a.k = k;
    a.rp = g->out.rp;
    a.col = g->out.col;
    a.w = g->out.w;
    a.src = ws.src;
    a.tdist = ws.tdist;
    a.tsig = ws.tsig;
    a.abits = ws.abits[b];
    a.fbits = ws.fbits[b];
    a.abits_n = ws.abits[bn];
    a.fbits_n = ws.fbits[bn];
    a.cnt = ws.fdist[0];
    a.zeta = ws.fsig[0];
    a.q = ws.fsig[1];
    a.step = ws.fdist[1];
    a.lam = ws.lam;
    a.pd = ws.pd;
    a.pm = ws.pm;
    a.ctr = ws.counters + (size_t)(k % kCounterRing) * 4 * kCounterSlots;
    a.nwords = (g->n + 31) / 32;
    a.clear_bits = ws.abits[b];
    a.clear_ctr = ws.counters + (size_t)((k + 1) % kCounterRing) * 4 * kCounterSlots;
    return a;
}

void launch_bwd_count(mfbc_graph *g, int ncg, hipStream_t s, hipEvent_t *ev) {
    Workspace &ws = g->ws;
    // the counting product writes B_0 into buffer 0: clear its bitmap and
    // this product's counters first
    const int nwords = (g->n + 31) / 32;
    hipMemsetAsync(ws.abits[0], 0, (size_t)nwords * ncg * 4, s);
    hipMemsetAsync(ws.abits[1], 0, (size_t)nwords * ncg * 4, s);
    hipMemsetAsync(ws.counters, 0, sizeof(unsigned long long) * kCounterRing * 4 * kCounterSlots, s);
    BwdArgs a = bwd_args(g, ncg, 0);
    if (ev) hipEventRecord(ev[0], s);
    const size_t waves = (size_t)a.ntasks * ncg;
    const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
    if (g->out.w)
        hipLaunchKernelGGL(k_bwd_count<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_bwd_count<false>, dim3(grid), dim3(kBlock), 0, s, a);
    int mgrid = blocks_for((size_t)a.nhubs * ncg, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_bwd_count_merge, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev) {
        hipEventRecord(ev[1], s);
        hipEventRecord(ev[2], s);
    }
}

void launch_bwd_product(mfbc_graph *g, int ncg, int k, hipStream_t s, hipEvent_t *ev) {
    BwdArgs a = bwd_args(g, ncg, k);
    if (ev) hipEventRecord(ev[0], s);
    const size_t waves = (size_t)a.ntasks * ncg;
    const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
    if (g->out.w)
        hipLaunchKernelGGL(k_bwd_pull<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_bwd_pull<false>, dim3(grid), dim3(kBlock), 0, s, a);
    if (ev) hipEventRecord(ev[1], s);
    int mgrid = blocks_for((size_t)a.nhubs * ncg, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_bwd_merge, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev) hipEventRecord(ev[2], s);
}

void launch_lambda_zero(mfbc_graph *g, int ncg, hipStream_t s) {
    const size_t total = (size_t)ncg * g->n;
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(total, 256, 65536)), dim3(256), 0, s, g->ws.lam,
                       total);
}

void launch_lambda_reduce(mfbc_graph *g, int ncg, double *d_bc, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_reduce, dim3(blocks_for(g->n, 256)), dim3(256), 0, s, g->ws.lam,
                       ncg, g->n, d_bc);
}

void launch_export_forward(mfbc_graph *g, int ncg, int nb, int32_t *d_dist, double *d_sigma,
                           uint64_t *d_fmask, hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    hipLaunchKernelGGL(k_tiles_to_rows<int32_t>, grid, dim3(kBlock), 0, s, g->ws.tdist, d_dist,
                       g->n, nb);
    hipLaunchKernelGGL(k_tiles_to_rows<double>, grid, dim3(kBlock), 0, s, g->ws.tsig, d_sigma,
                       g->n, nb);
    if (d_fmask)
        hipLaunchKernelGGL(k_tiles_to_rows<uint64_t>, grid, dim3(kBlock), 0, s,
                           (const uint64_t *)g->ws.fmask, d_fmask, g->n, nb);
}

void launch_import_forward(mfbc_graph *g, int ncg, int nb, const int32_t *d_dist,
                           const double *d_sigma, hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    hipLaunchKernelGGL(k_rows_to_tiles<int32_t>, grid, dim3(kBlock), 0, s, d_dist, g->ws.tdist,
                       g->n, nb, (int32_t)kInf);
    hipLaunchKernelGGL(k_rows_to_tiles<double>, grid, dim3(kBlock), 0, s, d_sigma, g->ws.tsig,
                       g->n, nb, 0.0);
}

void launch_export_backward(mfbc_graph *g, int ncg, int nb, double *d_delta, int32_t *d_step,
                            hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    hipLaunchKernelGGL(k_delta_rows, grid, dim3(kBlock), 0, s, (const double *)g->ws.fsig[0],
                       (const double *)g->ws.tsig, (const int32_t *)g->ws.tdist,
                       (const int32_t *)g->ws.src, d_delta, g->n, nb);
    if (d_step)
        hipLaunchKernelGGL(k_tiles_to_rows<int32_t>, grid, dim3(kBlock), 0, s,
                           (const int32_t *)g->ws.fdist[1], d_step, g->n, nb);
}

}  // namespace mfbc
