// The generalised product of Section 3, C = F (+).f A (a commutative monoid
// (+) on the outputs, an action f of an arc on an input entry), over one
// Task in pull form: the output at vertex v is the (+)-reduction, over the
// arcs u -> v whose source u is in the frontier, of f(F(u), w(u, v)); then
// T := T (+) C at v and the next frontier (the entries that C changed, in
// the sense of the algebra) are formed.  Every product of this shape runs
// through these functions -- MFBF's multpaths product (Algorithm 1),
// MFBr's backward product (Algorithm 2; both in products.h) and the monoid
// fixpoints (monoid.hip) -- with the algebra, the value type and the tile
// layout supplied by a policy P:
//
//   P::AM, P::U           arc format (see ArcSrc); active arcs per batch
//   P::H                  hub-slice partials in flight in the merge
//   P::Row                a lane's entries of one frontier row (every column
//                         group the wave holds)
//   P::Acc                the running (+)-reduction for the open owner
//   P::Own                the owner's T entries, loaded with its first candidate
//   p.bits, p.bits_n      activity bitmaps of the frontier read and written
//   p.absent(), p.none()  Row / Own placeholders
//   P::Tag, p.tag(u, e), p.live(tag)
//                         a per-arc payload computed by the lane holding arc
//                         e (source u, in the frontier) and whether the arc
//                         contributes to any lane: a product whose action
//                         is masked per lane (MFBr's stored shortest-path
//                         DAG) skips arcs that feed no lane
//   p.gather(u, tag, j)   frontier row of vertex u (this lane) for the arc held
//                         by lane j, whose tag is `tag` (read with readlane)
//   p.own(v0, o)          T at owner v0 + o (this lane; v0 = the task's first row)
//   p.batch(rows, us)     after a batch's gathers (e.g. side arrays read together)
//   p.reset(acc)          acc := the identity of (+)
//   p.fold(acc, row, w, u)  acc := acc (+) f(row, w)
//   p.finish(v, acc, own) T := T (+) acc at v, next frontier row; returns the
//                         lanes in the next frontier (any group)
//   p.store(part, acc), p.load(slot), p.merge(acc, part), p.finish_hub(v, acc)
//                         partials of a split (hub) row and their combination
//   P::kEveryRow, p.idle(v)  when set, every row of a run without a
//                         candidate is visited too (MFBr clears its frontier
//                         lane masks there)
//
// PullDefaults supplies the optional members (no tag, nothing masked, no
// batch hook, only rows with candidates visited).
//
// The task's arcs are read 64 at a time (the next 64 in flight while the
// current ones are processed); the arcs whose source is active are taken U
// at a time in arc order, whatever rows they belong to, and their row
// gathers -- plus the T row of every owner that starts in the batch -- are
// issued together, so one memory round trip serves several short rows.  The
// batch is then folded in arc order, each owner being finished when the next
// arc belongs to a later one.  A slice of a hub row has one owner and leaves
// a partial, combined with the other slices in slice order by pull_hub.
#pragma once

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

// The same in two halves, for loads issued a chunk ahead: load_arc_raw only
// loads (so the load stays in flight until decode_arc first needs it; a
// decode next to the load would wait for it there), decode_arc unpacks.
template <int AM>
__device__ __forceinline__ void load_arc_raw(const ArcSrc &s, int64_t e, uint32_t &r0, uint32_t &r1) {
    if (AM == 1) {
        r0 = s.pk[e];
    } else {
        r0 = (uint32_t)s.col[e];
        if (AM == 2) r1 = (uint32_t)s.w[e];
    }
}

template <int AM>
__device__ __forceinline__ void decode_arc(const ArcSrc &s, uint32_t r0, uint32_t r1, int &u, int &wt) {
    if (AM == 1) {
        u = (int)(r0 & s.cmask);
        wt = (int)(r0 >> s.cb);
    } else {
        u = (int)r0;
        wt = AM == 2 ? (int)r1 : 1;
    }
}

struct PullDefaults {
    struct Tag {};
    static constexpr bool kEveryRow = false;
    __device__ __forceinline__ Tag tag(int, int64_t) const { return Tag{}; }
    __device__ __forceinline__ bool live(const Tag &) const { return true; }
    __device__ __forceinline__ void idle(int) const {}
};

template <class P>
__device__ __forceinline__ void pull_task(P &p, const Task *tp, const int64_t *rp, const ArcSrc &arcs) {
    constexpr int U = P::U;
    constexpr int AM = P::AM;
    const int lane = threadIdx.x & (kWave - 1);
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const uint32_t *Ab = p.bits;
    // end of each owner's arcs, one owner per lane (a run has at most 64
    // rows), relative to the task's first arc (a task's arcs fit 32 bits);
    // the owner of arc e is the number of rows ending at or before e.
    const int rend = (hub < 0 && v0 + lane < v1) ? (int)(rp[v0 + lane + 1] - e0) : INT32_MAX;
    int cur = -1;            // owner (offset from v0) of the open reduction
    typename P::Acc acc;
    typename P::Own own = p.none();
    p.reset(acc);
    uint64_t run_act = 0;
    uint32_t rn0 = 0, rn1 = 1;          // this lane's arc of the next chunk, not yet decoded
    if (e0 + lane < e1) load_arc_raw<AM>(arcs, e0 + lane, rn0, rn1);
    for (int64_t e = e0; e < e1; e += kWave) {
        const int64_t my = e + lane;
        const int eoff = (int)(e - e0);
        int u, wt;
        decode_arc<AM>(arcs, rn0, rn1, u, wt);
        bool act = my < e1 && ((Ab[u >> 5] >> (u & 31)) & 1u);
        typename P::Tag tg{};
        if (act) {
            tg = p.tag(u, my);
            act = p.live(tg);
        }
        // the next chunk's arcs: packed or two-array arcs (AM != 0) are
        // requested after this chunk's first gathers, so that the gathers
        // do not wait for them (1% on the weighted forward product); plain
        // columns (AM = 0) here, where it costs the kernel no register
        bool pf = AM == 0;
        if (AM == 0 && my + kWave < e1) load_arc_raw<AM>(arcs, my + kWave, rn0, rn1);
        // Per active arc the wave spends most of its scalar instructions here,
        // and the scalar unit is the kernel's busiest pipe after memory: the
        // batch takes min(U, active) arcs by count, so that each needs one
        // find-first-bit and one bit clear, not a test of an empty mask.
        uint64_t am = ballot(act);
        int na = __popcll(am);
        while (na > 0) {
            int ow[U], wk[U], uk[U];
            typename P::Row rk[U];
            typename P::Own on[U];
            int prev = cur;
#pragma unroll
            for (int k = 0; k < U; k++) {
                ow[k] = -1;
                uk[k] = 0;
                wk[k] = 0;
                rk[k] = p.absent();
                on[k] = p.none();
                if (k < na) {
                    const int j = __builtin_ctzll(am);      // am != 0 here
                    am &= ~(1ull << j);
                    uk[k] = rdlane(u, j);
                    wk[k] = AM ? rdlane(wt, j) : 1;
                    rk[k] = p.gather(uk[k], tg, j);
                    ow[k] = __popcll(ballot(rend <= eoff + j));
                    // (a hub slice's single owner is loaded too, and not used)
                    if (ow[k] != prev) on[k] = p.own(v0, ow[k]);
                    prev = ow[k];
                }
            }
            na -= U;
            if (!pf) {
                if (my + kWave < e1) load_arc_raw<AM>(arcs, my + kWave, rn0, rn1);
                pf = true;
            }
            p.batch(rk, uk);
#pragma unroll
            for (int k = 0; k < U; k++) {
                if (ow[k] >= 0) {
                    if (ow[k] != cur) {
                        if (cur >= 0 && hub < 0 && p.finish(v0 + cur, acc, own)) run_act |= 1ull << cur;
                        if constexpr (P::kEveryRow)
                            if (hub < 0)
                                for (int o = cur + 1; o < ow[k]; o++) p.idle(v0 + o);
                        cur = ow[k];
                        p.reset(acc);
                        own = on[k];
                    }
                    p.fold(acc, rk[k], wk[k], uk[k]);
                }
            }
        }
        if (!pf && my + kWave < e1) load_arc_raw<AM>(arcs, my + kWave, rn0, rn1);
    }
    if (hub < 0) {
        if (cur >= 0 && p.finish(v0 + cur, acc, own)) run_act |= 1ull << cur;
        if constexpr (P::kEveryRow)
            for (int o = cur + 1; o < v1 - v0; o++) p.idle(v0 + o);
        if (lane == 0 && run_act) or_run_bits(p.bits_n, v0, run_act);
    } else {
        p.store(part, acc);
    }
}

// The same product in owner order: the task's rows are taken one after
// another and the batch of U active arcs is drawn from the current row only,
// the owner's T entries loaded with the batch's gathers.  Fewer registers
// than batches across owners (the batch needs no owner index per arc), for
// products whose rows are finished often without a candidate (P::kEveryRow)
// and whose per-arc masks already skip the arcs that feed no lane.
__device__ __forceinline__ uint64_t owner_mask(int64_t e, int64_t vend) {
    const int64_t lim = vend - e;
    return lim >= kWave ? ~0ull : (lim <= 0 ? 0ull : ((1ull << lim) - 1ull));
}

template <class P>
__device__ __forceinline__ void pull_task_owner(P &p, const Task *tp, const int64_t *rp, const ArcSrc &arcs) {
    constexpr int U = P::U;
    constexpr int AM = P::AM;
    const int lane = threadIdx.x & (kWave - 1);
    const int v0 = uni(tp->v0), v1 = uni(tp->v1), hub = uni(tp->hub), part = uni(tp->part);
    const int64_t e0 = uni64(tp->e0), e1 = uni64(tp->e1);
    const uint32_t *Ab = p.bits;
    int x = v0;
    int64_t vend = hub >= 0 ? e1 : rp[v0 + 1];
    bool loaded = false;
    typename P::Acc acc;
    typename P::Own own = p.none();
    p.reset(acc);
    uint64_t run_act = 0;
    auto close = [&]() {
        if (loaded) {
            if (p.finish(x, acc, own)) run_act |= 1ull << (x - v0);
        } else if constexpr (P::kEveryRow) {
            p.idle(x);
        }
        loaded = false;
        p.reset(acc);
    };
    for (int64_t e = e0; e < e1; e += kWave) {
        const int64_t my = e + lane;
        int y = 0, wt = 1;
        typename P::Tag tg{};
        bool act = false;
        if (my < e1) {
            load_arc<AM>(arcs, my, y, wt);
            if ((Ab[y >> 5] >> (y & 31)) & 1u) {
                tg = p.tag(y, my);
                act = p.live(tg);
            }
        }
        uint64_t am = ballot(act);
        while (am) {
            const int j0 = __ffsll((unsigned long long)am) - 1;
            if (hub < 0) {
                while (e + j0 >= vend) {
                    close();
                    ++x;
                    vend = rp[x + 1];
                }
            }
            uint64_t cand = am & owner_mask(e, vend);
            int wk[U], uk[U];
            typename P::Row rk[U];
#pragma unroll
            for (int k = 0; k < U; k++) {
                rk[k] = p.absent();
                uk[k] = 0;
                wk[k] = 0;
                if (cand) {
                    const int j = __ffsll((unsigned long long)cand) - 1;
                    cand &= cand - 1;
                    am &= ~(1ull << j);
                    uk[k] = rdlane(y, j);
                    wk[k] = AM ? rdlane(wt, j) : 1;
                    rk[k] = p.gather(uk[k], tg, j);
                }
            }
            if (!loaded) {
                own = p.own(v0, x - v0);
                loaded = true;
            }
            p.batch(rk, uk);
#pragma unroll
            for (int k = 0; k < U; k++) p.fold(acc, rk[k], wk[k], uk[k]);
        }
    }
    if (hub < 0) {
        while (x < v1) {
            close();
            ++x;
        }
        if (lane == 0 && run_act) or_run_bits(p.bits_n, v0, run_act);
    } else {
        p.store(part, acc);
    }
}

// Combine the slices of split row h in slice order (P::H partials in
// flight) and finish the row.
template <class P>
__device__ __forceinline__ void pull_hub(P &p, const Hub *hp) {
    constexpr int H = P::H;
    const int lane = threadIdx.x & (kWave - 1);
    const int v = uni(hp->v), first = uni(hp->first), np = uni(hp->nparts);
    typename P::Acc acc;
    p.reset(acc);
    for (int s0 = first; s0 < first + np; s0 += H) {
        typename P::Acc pt[H];
#pragma unroll
        for (int k = 0; k < H; k++) {
            if (s0 + k < first + np) pt[k] = p.load(s0 + k);
            else p.reset(pt[k]);
        }
#pragma unroll
        for (int k = 0; k < H; k++) p.merge(acc, pt[k]);
    }
    if (p.finish_hub(v, acc) && lane == 0) atomicOr(p.bits_n + (v >> 5), 1u << (v & 31));
}

}  // namespace
}  // namespace mfbc
