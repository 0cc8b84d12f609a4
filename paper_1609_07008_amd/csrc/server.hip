// Served form: continuous batching of source columns over a resident graph.
//
// A server owns `width` source columns (a multiple of 64) of one graph.  Each
// column holds one source of some request and moves through the phases FWD
// (Algorithm 1's loop), CNT (the counting product of Algorithm 2), BWD
// (Algorithm 2's loop), DONE (ready to harvest), FREE.  Column s of every
// product depends only on column s of its frontier (the product's output
// column is a function of the same input column, Section 3), so columns can
// join and leave at step boundaries while other columns are mid-loop: one
// step runs one counting product (every CNT column) and then R rounds of one
// forward product (every FWD column) and one backward product (every BWD or
// just-counted column), each launched only over the pairs of 64-column
// groups that have columns in it, with the same paired kernels as the plain
// path.  A product whose predecessor in the step produced nothing skips
// itself on the device, and frontiers only shrink to empty, so phases are
// updated from the step's last round: R products cost one round trip to the
// host.
//
// The unit of admission is the pair of 64-column groups (2p, 2p+1; the last
// pair may hold a single group): a product's cost per pair is set by the
// union of its lanes' frontiers and its full pass over the arcs in the
// counting product, whatever the number of lanes, so a pair admits new
// sources only when all of its columns are free (from several requests at
// once, until the next step is launched), leaves the forward loop when every
// one of its lanes has an empty frontier, and runs one counting product --
// exactly the per-batch schedule of the plain path, while different pairs
// sit in different phases.  Columns that finish the backward loop become
// DONE one by one.  The forward and backward states have separate buffers,
// since one step holds pairs in both loops.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "products.h"

namespace mfbc {
namespace {

enum Phase : uint8_t { kFree = 0, kFwd = 1, kCnt = 2, kBwd = 3, kDone = 4 };

constexpr int kMaxRounds = 8;              // product rounds per step, at most

// Counters of round r of product kind k (0 forward, 1 backward, 2 counting).
inline size_t ctr_slot(int k, int r) { return ((size_t)k * (kMaxRounds + 1) + r) * 4 * kCounterSlots; }
constexpr size_t kCtrWords = (size_t)3 * (kMaxRounds + 1) * 4 * kCounterSlots;

// New columns: T = (INF, 0) and backward frontier bits cleared.  Their
// counters and zeta need no reset: the counting product writes both for every
// vertex and every lane of the counted pair before a backward product reads
// them.
__global__ void k_srv_reset_cols(int n, const uint64_t *newmask, int32_t *tdist, double *tsig,
                                 uint64_t *bb0, uint64_t *bb1) {
    const int cg = blockIdx.y;
    const uint64_t m = newmask[cg];
    if (!m) return;
    const int lane = threadIdx.x & (kWave - 1);
    const bool mine = (m >> lane) & 1ull;
    const int v0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int stride = (gridDim.x * blockDim.x) >> 6;
    for (int v = v0; v < n; v += stride) {
        const size_t idx = ((size_t)cg * n + v) * kWave + lane;
        if (mine) {
            tdist[idx] = kInf;
            tsig[idx] = 0.0;
        }
        if (lane == 0) {
            // backward lane masks are interleaved per pair of groups
            const size_t i = ((size_t)(cg >> 1) * n + v) * 2 + (cg & 1);
            bb0[i] &= ~m;
            bb1[i] &= ~m;
        }
    }
}

// Pair rows (groups 2q and 2q+1, kWide = 2 entries per lane) of new sources
// that are not yet in the current forward frontier start with every lane of
// both groups absent (no lane of the pair is in the frontier there).
__global__ void k_srv_seed_rows(int n, int nwords, const int32_t *cols, int count,
                                const int32_t *src, uint32_t *ftup, const uint32_t *abits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int c = cols[i], v = src[c], q = c / (kWave * kWide);
    if ((abits[(size_t)q * nwords + (v >> 5)] >> (v & 31)) & 1u) return;
    const size_t row = ((size_t)q * n + v) * kWave * kWide;
    for (int l = 0; l < kWave * kWide; l++) ftup[row + l] = kSent;
}

__global__ void k_srv_seed(int n, int nwords, const int32_t *cols, int count, const int32_t *src,
                           int32_t *tdist, double *tsig, uint32_t *ftup, uint32_t *abits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int c = cols[i], v = src[c], cg = c / kWave, lane = c % kWave, q = cg / kWide;
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    tdist[idx] = 0;
    tsig[idx] = 1.0;
    ftup[(((size_t)q * n + v) * kWave + lane) * kWide + (cg % kWide)] = 1u;
    atomicOr(abits + (size_t)q * nwords + (v >> 5), 1u << (v & 31));
}

// dest_i[v] += delta(column cols[i], v) for every listed column.  The list
// arrives grouped by column group (entries of group g at [gofs[g],
// gofs[g+1]), each group's in list order).  A block takes 64 caller vertices;
// for every group with listed columns it stages delta of the group's 64
// lanes at those vertices in LDS -- coalesced 64-lane rows of the tiles,
// gathered through `perm` -- then one thread per vertex adds the group's
// columns in order, with one read-modify-write per run of consecutive
// entries that share a destination.  A destination shared by several columns
// is thus updated group by group, in list order within a group.
__global__ __launch_bounds__(256) void k_srv_harvest_bc(int n, int ncg, const int32_t *cols,
                                                        const int32_t *gofs, const int32_t *src,
                                                        double *const *dest, const int32_t *tdist,
                                                        const double *tsig, const double *zeta,
                                                        const int32_t *perm) {
    __shared__ double sh[64][65];
    const int v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int g = 0; g < ncg; g++) {
        const int e0 = gofs[g], e1 = gofs[g + 1];
        if (e0 == e1) continue;
        __syncthreads();                 // the previous group's tile is consumed
        const int s = src[g * kWave + c];
        for (int r = r0; r < 64; r += 4) {
            const int v = v0 + r;
            double dv = 0.0;
            if (v < n) {
                const int d = perm ? perm[v] : v;
                const size_t idx = ((size_t)g * n + d) * kWave + c;
                if (tdist[idx] != kInf && d != s) dv = zeta[idx] * tsig[idx];
            }
            sh[r][c] = dv;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int v = v0 + threadIdx.x;
            if (v < n) {
                double *cur = nullptr;
                double acc = 0.0;
                for (int e = e0; e < e1; e++) {
                    double *p = dest[e];
                    const double x = sh[threadIdx.x][cols[e] & (kWave - 1)];
                    if (p != cur) {
                        if (cur) cur[v] += acc;
                        cur = p;
                        acc = x;
                    } else {
                        acc += x;
                    }
                }
                if (cur) cur[v] += acc;
            }
        }
    }
}

// out_i[t] = delta(column cols[i], targets[t]) (targets in caller ids).
__global__ void k_srv_harvest_dep(int n, const int32_t *cols, int count, const int32_t *src,
                                  const int32_t *targets, int ntargets, double *const *out,
                                  const int32_t *tdist, const double *tsig, const double *zeta,
                                  const int32_t *perm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count * ntargets) return;
    const int i = k / ntargets, t = k % ntargets;
    const int c = cols[i], cg = c / kWave, lane = c % kWave;
    const int v = perm ? perm[targets[t]] : targets[t];
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    out[i][t] = (tdist[idx] != kInf && v != src[c]) ? zeta[idx] * tsig[idx] : 0.0;
}

// tau of the listed pairs of groups interleaved per lane in 16 bits a group
// (the paired counting product's input): tau2[q][v][lane] = (group 2q,
// group 2q+1) at (v, lane), packed by pack_tau16; *full (cleared by
// k_srv_clear_flag before) is set when a finite tau does not fit.
__global__ void k_srv_pair_tau(const int32_t *tdist, uint32_t *tau2, size_t plane, int ncg,
                               const int32_t *plist, int np, int32_t *full) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t total = (size_t)np * plane;
    bool big = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const size_t k = i / plane, r = i - k * plane;
        const int q = plist[k];
        const int x = tdist[(size_t)(2 * q) * plane + r];
        const int y = 2 * q + 1 < ncg ? tdist[(size_t)(2 * q + 1) * plane + r] : kInf;
        big |= tau16_big(x) || tau16_big(y);
        tau2[(size_t)q * plane + r] = pack_tau16(x, y);
    }
    if (big) *full = 1;
}

__global__ void k_srv_clear_flag(int32_t *flag) {
    if (threadIdx.x == 0) *flag = 0;
}

inline int nblocks(size_t work, int per, int cap = 1 << 20) {
    size_t b = (work + per - 1) / per;
    return (int)std::max<size_t>(1, std::min<size_t>(b, (size_t)cap));
}

}  // namespace
}  // namespace mfbc

using namespace mfbc;

struct mfbc_server {
    mfbc_graph *g = nullptr;
    int width = 0, ncg = 0, nwords = 0;
    int npair = 0;                          // forward pairs (groups 2p, 2p+1; the last may be
                                            // half padding, whose tiles exist but hold no column)
    int cur_f = 0, cur_b = 0, kfwd = 0, kbwd = 0;
    int32_t slot_cap = 0;                   // hub partial slots the server's pd/pm hold
    int32_t *tdist = nullptr;
    double *tsig = nullptr;
    uint32_t *ftup[2] = {nullptr, nullptr};
    double *fsig[2] = {nullptr, nullptr};
    uint32_t *abf[2] = {nullptr, nullptr};
    int32_t *cnt = nullptr;
    double *zeta = nullptr, *q = nullptr;
    uint64_t *bb[2] = {nullptr, nullptr};
    uint32_t *abb[2] = {nullptr, nullptr};
    int32_t *pd = nullptr;
    double *pm = nullptr;
    int32_t *src = nullptr;
    int rounds = 0;                         // rounds of products per step (0: by graph size)
    int nrounds = 1;                        // rounds of the step in flight
    unsigned long long *ctr = nullptr;      // [kind][round][4][32] product counters: kind 0
                                            // forward, 1 backward, 2 counting (one round);
                                            // round kMaxRounds is the last merge's clear target
    unsigned long long *colmask = nullptr;  // [round][3][32][ncg]: forward, counting, backward
    uint64_t *cmask = nullptr;              // [ncg] counting mask
    uint64_t *newmask = nullptr;            // [ncg] columns being admitted
    int32_t *cglists = nullptr;             // [4][ncg]: pairs with forward / backward /
                                            // counting columns this step, counting groups
    uint32_t *tau2 = nullptr;               // [npair][n][64] 16-bit tau pairs of the counted pairs
    int32_t *flags = nullptr;               // [0] path count overflow, [1] tau beyond 16 bits
    uint64_t *dag = nullptr;                // [ncg][arcs] shortest-path lane masks of each
                                            // group's cohort (counting product writes)
    char *meta = nullptr;                   // staging for harvest/admit lists
    size_t meta_bytes = 0;
    unsigned long long *h_colmask = nullptr;  // pinned
    hipEvent_t done_ev = nullptr;             // recorded at the end of a launched step
    std::vector<int32_t> h_src;
    std::vector<uint8_t> phase;
    std::vector<uint8_t> ran_f, ran_b, ran_c; // columns taking part in the launched step
    std::vector<uint8_t> open;                // [npair] pairs admitting since the last launch
    int32_t *h_stage = nullptr;               // pinned: [4][ncg] lists, then [ncg] masks
    int32_t *h_flags = nullptr;               // pinned copy of flags[0] (path count overflow)
    bool launched = false, any_f = false, any_b = false, any_c = false;
};

namespace {

int sfail(int code, const std::string &m) { return set_error(code, m); }

template <typename T>
int salloc(T **p, size_t count) {
    *p = nullptr;
    if (hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return MFBC_ENOMEM;
    }
    return MFBC_OK;
}

template <typename T>
void sfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_server(mfbc_server *s) {
    sfree(s->tdist);
    sfree(s->tsig);
    for (int b = 0; b < 2; b++) {
        sfree(s->ftup[b]);
        sfree(s->fsig[b]);
        sfree(s->abf[b]);
        sfree(s->bb[b]);
        sfree(s->abb[b]);
    }
    sfree(s->cnt);
    sfree(s->zeta);
    sfree(s->q);
    sfree(s->pd);
    sfree(s->pm);
    sfree(s->src);
    sfree(s->ctr);
    sfree(s->colmask);
    sfree(s->cmask);
    sfree(s->newmask);
    sfree(s->cglists);
    sfree(s->tau2);
    sfree(s->flags);
    sfree(s->dag);
    sfree(s->meta);
    if (s->h_colmask) (void)hipHostFree(s->h_colmask);
    s->h_colmask = nullptr;
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    s->h_stage = nullptr;
    if (s->h_flags) (void)hipHostFree(s->h_flags);
    s->h_flags = nullptr;
    if (s->done_ev) (void)hipEventDestroy(s->done_ev);
    s->done_ev = nullptr;
}

ArcSrc srv_arc_src(const Csr &c) {
    ArcSrc r{};
    r.col = c.col;
    r.w = c.w;
    r.pk = c.pk;
    r.cb = c.cb;
    r.cmask = c.cb >= 32 ? 0xffffffffu : ((1u << c.cb) - 1u);
    return r;
}

int srv_mode(const Csr &c) { return c.w == nullptr ? 0 : (c.pk ? 1 : 2); }

int stage(mfbc_server *s, size_t bytes) {
    if (s->meta_bytes >= bytes) return MFBC_OK;
    sfree(s->meta);
    s->meta_bytes = 0;
    if (salloc(&s->meta, bytes)) return sfail(MFBC_ENOMEM, "staging allocation failed");
    s->meta_bytes = bytes;
    return MFBC_OK;
}

// Rounds per step by default: eight on every graph (measured on R-MAT scales
// 14..20: fewer round trips cost more than the later admission of new
// sources).
int server_rounds(const mfbc_graph *g) {
    (void)g;
    return kMaxRounds;
}

#define SHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return sfail(MFBC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

int mfbc_server_footprint(const mfbc_graph *g, int32_t width, int64_t *bytes) {
    if (!g || !bytes || width < 64 || width % 64) return sfail(MFBC_EINVAL, "bad arguments");
    const int64_t n = g->n, ncg = width / 64, ncg2 = (ncg + 1) & ~1;
    const int64_t slots = std::max(g->plan_in.nslots, g->plan_out.nslots);
    const int64_t nw = (n + 31) / 32;
    // tiles: T (4 + 8), frontier tuples (2 x (4 + 8)), counters, zeta, q
    // (4 + 8 + 8) and the counting product's 16-bit tau copy (2), per (column, vertex)
    *bytes = n * 64 * ncg2 * (4 + 8 + 2 * 4 + 2 * 8 + 4 + 8 + 8 + 2) + 2 * ncg2 * n * 8 +
             4 * ncg * nw * 4 + slots * 64 * ncg2 * 12 + ncg * std::max<int64_t>(g->arcs, 1) * 8;
    return MFBC_OK;
}

int mfbc_server_create(mfbc_graph *g, int32_t width, mfbc_server **out) {
    if (!g || !out) return sfail(MFBC_EINVAL, "NULL argument");
    if (width < 64 || width % 64) return sfail(MFBC_EINVAL, "width must be a positive multiple of 64");
    *out = nullptr;
    mfbc_server *s = new (std::nothrow) mfbc_server();
    if (!s) return sfail(MFBC_ENOMEM, "host allocation failed");
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(g->device);
    s->g = g;
    s->width = width;
    s->ncg = width / 64;
    s->npair = (s->ncg + kWide - 1) / kWide;
    s->nwords = (g->n + 31) / 32;
    // per-(column, vertex) tiles and hub slots cover whole pairs
    const size_t n = (size_t)g->n, ncg = (size_t)s->ncg, ncg2 = (size_t)s->npair * kWide;
    const size_t tile = n * kWave * ncg2;
    const size_t slots = (size_t)std::max(g->plan_in.nslots, g->plan_out.nslots) * kWave * ncg2;
    int rc = MFBC_OK;
    if (salloc(&s->tdist, tile) || salloc(&s->tsig, tile) || salloc(&s->ftup[0], tile) ||
        salloc(&s->ftup[1], tile) || salloc(&s->fsig[0], tile) || salloc(&s->fsig[1], tile) ||
        salloc(&s->abf[0], ncg * s->nwords) || salloc(&s->abf[1], ncg * s->nwords) ||
        salloc(&s->cnt, tile) || salloc(&s->zeta, tile) || salloc(&s->q, tile) ||
        salloc(&s->bb[0], ncg2 * n) || salloc(&s->bb[1], ncg2 * n) || salloc(&s->tau2, tile / 2) ||
        salloc(&s->abb[0], ncg * s->nwords) || salloc(&s->abb[1], ncg * s->nwords) ||
        salloc(&s->pd, slots) || salloc(&s->pm, slots) || salloc(&s->src, (size_t)width) ||
        salloc(&s->ctr, kCtrWords) || salloc(&s->colmask, (size_t)kMaxRounds * 3 * 32 * ncg) ||
        salloc(&s->cmask, ncg) || salloc(&s->newmask, ncg) || salloc(&s->cglists, 4 * ncg) ||
        salloc(&s->flags, 4) || salloc(&s->dag, ncg * (size_t)std::max<int64_t>(g->arcs, 1)))
        rc = MFBC_ENOMEM;
    if (!rc && hipHostMalloc((void **)&s->h_colmask, 2 * 3 * 32 * ncg * 8) != hipSuccess) rc = MFBC_ENOMEM;
    if (!rc && hipHostMalloc((void **)&s->h_stage, 4 * ncg * 4 + ncg * 8) != hipSuccess) rc = MFBC_ENOMEM;
    if (!rc && hipHostMalloc((void **)&s->h_flags, 16) != hipSuccess) rc = MFBC_ENOMEM;
    if (!rc && hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming) != hipSuccess)
        rc = MFBC_EDEVICE;
    if (!rc) {
        // every column free: counters off, no frontier anywhere
        hipStream_t st = nullptr;
        if (hipMemsetAsync(s->cnt, 0xff, tile * 4, st) != hipSuccess ||
            hipMemsetAsync(s->bb[0], 0, ncg2 * n * 8, st) != hipSuccess ||
            hipMemsetAsync(s->bb[1], 0, ncg2 * n * 8, st) != hipSuccess ||
            hipMemsetAsync(s->abf[0], 0, ncg * s->nwords * 4, st) != hipSuccess ||
            hipMemsetAsync(s->abf[1], 0, ncg * s->nwords * 4, st) != hipSuccess ||
            hipMemsetAsync(s->abb[0], 0, ncg * s->nwords * 4, st) != hipSuccess ||
            hipMemsetAsync(s->abb[1], 0, ncg * s->nwords * 4, st) != hipSuccess ||
            hipMemsetAsync(s->src, 0xff, (size_t)width * 4, st) != hipSuccess ||
            hipMemsetAsync(s->flags, 0, 16, st) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            rc = MFBC_EDEVICE;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (rc) {
        free_server(s);
        delete s;
        return sfail(rc, rc == MFBC_ENOMEM ? "device allocation failed" : "initialisation failed");
    }
    s->slot_cap = std::max(g->plan_in.nslots, g->plan_out.nslots);
    g->servers++;              // the graph's plan is frozen while servers are attached
    s->h_src.assign((size_t)width, -1);
    s->phase.assign((size_t)width, kFree);
    s->ran_f.assign((size_t)width, 0);
    s->ran_b.assign((size_t)width, 0);
    s->ran_c.assign((size_t)width, 0);
    s->open.assign((size_t)s->npair, 0);
    *out = s;
    return MFBC_OK;
}

int mfbc_server_free(mfbc_server *s) {
    if (!s) return MFBC_OK;
    (void)hipDeviceSynchronize();
    if (s->g && s->g->servers > 0) s->g->servers--;
    free_server(s);
    delete s;
    return MFBC_OK;
}

// A pair of groups admits sources if it was opened since the last launch or
// if every one of its columns is free.
static bool pair_admits(const mfbc_server *s, int q) {
    if (s->open[(size_t)q]) return true;
    const int c0 = q * kWide * kWave, c1 = std::min(s->width, c0 + kWide * kWave);
    for (int c = c0; c < c1; c++)
        if (s->phase[(size_t)c] != kFree) return false;
    return true;
}

int mfbc_server_free_columns(const mfbc_server *s) {
    if (!s) return sfail(MFBC_EINVAL, "NULL server");
    int f = 0;
    for (int q = 0; q < s->npair; q++) {
        if (!pair_admits(s, q)) continue;
        const int c0 = q * kWide * kWave, c1 = std::min(s->width, c0 + kWide * kWave);
        for (int c = c0; c < c1; c++) f += s->phase[(size_t)c] == kFree;
    }
    return f;
}

int mfbc_server_active_columns(const mfbc_server *s) {
    if (!s) return sfail(MFBC_EINVAL, "NULL server");
    int f = 0;
    for (uint8_t p : s->phase) f += p == kFwd || p == kCnt || p == kBwd;
    return f;
}

int mfbc_server_admit(mfbc_server *s, const int32_t *h_sources, int32_t count, int32_t *h_columns,
                      void *hip_stream) {
    if (!s || (count > 0 && (!h_sources || !h_columns))) return sfail(MFBC_EINVAL, "NULL argument");
    if (s->launched) return sfail(MFBC_EINVAL, "a step is in flight");
    if (count <= 0) return MFBC_OK;
    for (int i = 0; i < count; i++)
        if (h_sources[i] < 0 || h_sources[i] >= s->g->n) return sfail(MFBC_EINVAL, "source out of range");
    // fill the pairs opened since the last launch first, then whole free pairs
    std::vector<int32_t> cols;
    for (int pass = 0; pass < 2 && (int)cols.size() < count; pass++)
        for (int q = 0; q < s->npair && (int)cols.size() < count; q++) {
            if (pass == 0 ? !s->open[(size_t)q] : (s->open[(size_t)q] || !pair_admits(s, q)))
                continue;
            const int c1 = std::min(s->width, (q + 1) * kWide * kWave);
            for (int c = q * kWide * kWave; c < c1 && (int)cols.size() < count; c++)
                if (s->phase[(size_t)c] == kFree) cols.push_back(c);
        }
    if ((int)cols.size() < count) return sfail(MFBC_EINVAL, "not enough free columns");
    hipStream_t st = (hipStream_t)hip_stream;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->g->device);
    std::vector<uint64_t> nm((size_t)s->ncg, 0);
    for (int i = 0; i < count; i++) {
        const int c = cols[(size_t)i];
        h_columns[i] = c;
        // columns hold device vertex ids
        s->h_src[(size_t)c] = s->g->h_perm.empty() ? h_sources[i]
                                                   : s->g->h_perm[(size_t)h_sources[i]];
        s->phase[(size_t)c] = kFwd;
        s->open[(size_t)(c / (kWide * kWave))] = 1;
        nm[(size_t)(c / 64)] |= 1ull << (c % 64);
    }
    int rc = stage(s, (size_t)count * 4 + 256);
    if (rc) return rc;
    SHIP(hipMemcpyAsync(s->meta, cols.data(), (size_t)count * 4, hipMemcpyHostToDevice, st));
    SHIP(hipMemcpyAsync(s->newmask, nm.data(), (size_t)s->ncg * 8, hipMemcpyHostToDevice, st));
    SHIP(hipMemcpyAsync(s->src, s->h_src.data(), (size_t)s->width * 4, hipMemcpyHostToDevice, st));
    const int n = s->g->n;
    hipLaunchKernelGGL(k_srv_reset_cols, dim3(nblocks((size_t)n * 64, 256, 4096), s->ncg), dim3(256),
                       0, st, n, (const uint64_t *)s->newmask, s->tdist, s->tsig, s->bb[0], s->bb[1]);
    hipLaunchKernelGGL(k_srv_seed_rows, dim3(nblocks((size_t)count, 256)), dim3(256), 0, st, n,
                       s->nwords, (const int32_t *)s->meta, count, (const int32_t *)s->src,
                       s->ftup[s->cur_f], (const uint32_t *)s->abf[s->cur_f]);
    hipLaunchKernelGGL(k_srv_seed, dim3(nblocks((size_t)count, 256)), dim3(256), 0, st, n,
                       s->nwords, (const int32_t *)s->meta, count, (const int32_t *)s->src,
                       s->tdist, s->tsig, s->ftup[s->cur_f], s->abf[s->cur_f]);
    SHIP(hipGetLastError());
    SHIP(hipStreamSynchronize(st));
    if (prev >= 0) (void)hipSetDevice(prev);
    return MFBC_OK;
}

int mfbc_server_step_launch(mfbc_server *s, void *hip_stream) {
    if (!s) return sfail(MFBC_EINVAL, "NULL server");
    if (s->launched) return sfail(MFBC_EINVAL, "a step is already in flight");
    hipStream_t st = (hipStream_t)hip_stream;
    mfbc_graph *g = s->g;
    if (std::max(g->plan_in.nslots, g->plan_out.nslots) > s->slot_cap)
        return sfail(MFBC_EINVAL, "the graph's plan needs more hub partial slots than the server holds");
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(g->device);
    s->any_f = s->any_b = s->any_c = false;
    std::fill(s->open.begin(), s->open.end(), 0);   // admitted groups are now running
    uint64_t *cm = (uint64_t *)(s->h_stage + 4 * (size_t)s->ncg);   // after the four lists
    std::fill(cm, cm + s->ncg, 0ull);
    std::vector<uint8_t> gf((size_t)s->ncg, 0), gb((size_t)s->ncg, 0), gc((size_t)s->ncg, 0);
    for (int c = 0; c < s->width; c++) {
        const uint8_t p = s->phase[(size_t)c];
        s->ran_f[(size_t)c] = p == kFwd;
        s->ran_b[(size_t)c] = p == kBwd || p == kCnt;  // counted columns join this step's rounds
        s->ran_c[(size_t)c] = p == kCnt;
        s->any_f |= p == kFwd;
        s->any_b |= p == kBwd || p == kCnt;
        if (p == kFwd) gf[(size_t)(c / 64)] = 1;
        if (p == kBwd || p == kCnt) gb[(size_t)(c / 64)] = 1;
        if (p == kCnt) {
            s->any_c = true;
            gc[(size_t)(c / 64)] = 1;
            cm[(size_t)(c / 64)] |= 1ull << (c % 64);
        }
    }
    const size_t ncg = (size_t)s->ncg;
    // each product runs only over the pairs of groups that have columns in its
    // phase (a product's cost is per pair, whatever the number of columns):
    // lists of pairs for the forward, backward and counting products, and the
    // groups of the counted pairs (the counting product's hub merge)
    int32_t *lists = s->h_stage;
    int nf = 0, nbk = 0, nc = 0, ncgc = 0;
    for (int q = 0; q < s->npair; q++) {
        bool f = false, b = false, cc = false;
        for (int c = 0; c < kWide; c++) {
            const size_t g2 = (size_t)(q * kWide + c);
            if (g2 >= ncg) break;
            f |= gf[g2] != 0;
            b |= gb[g2] != 0;
            cc |= gc[g2] != 0;
        }
        if (f) lists[(size_t)nf++] = q;
        if (b) lists[ncg + (size_t)nbk++] = q;
        if (cc) {
            lists[2 * ncg + (size_t)nc++] = q;
            for (int c = 0; c < kWide && (size_t)(q * kWide + c) < ncg; c++)
                lists[3 * ncg + (size_t)ncgc++] = q * kWide + c;
        }
    }
    const int R = s->rounds > 0 ? s->rounds : server_rounds(g);
    s->nrounds = R;
    SHIP(hipMemcpyAsync(s->cglists, lists, 4 * ncg * 4, hipMemcpyHostToDevice, st));
    SHIP(hipMemsetAsync(s->colmask, 0, (size_t)R * 3 * 32 * ncg * 8, st));
    SHIP(hipMemsetAsync(s->ctr, 0, kCtrWords * 8, st));
    const int nw = s->nwords;
    const size_t cmw = 3 * 32 * ncg;                 // colmask words of one round
    BwdArgs c{};
    c.tasks = g->plan_out.tasks;
    c.hubs = g->plan_out.hubs;
    c.ntasks = g->plan_out.ntasks;
    c.nhubs = g->plan_out.nhubs;
    c.nslots = g->plan_out.nslots;
    c.ncg_all = s->ncg;
    c.nwide_all = s->npair;                          // backward state interleaved per pair
    c.n = g->n;
    c.nwords = nw;
    c.rp = g->out.rp;
    c.arcs = srv_arc_src(g->out);
    c.src = s->src;
    c.tdist = s->tdist;
    c.tsig = s->tsig;
    c.cnt = s->cnt;
    c.zeta = s->zeta;
    c.q = s->q;
    c.step = nullptr;
    c.lam = nullptr;
    c.pd = s->pd;
    c.pm = s->pm;
    c.tau2 = (const uint32_t *)s->tau2;
    c.tau_full = s->flags + 1;
    // the pair's columns reach the counting product together (cohort
    // admission), so its DAG masks are written whole and stay valid for its
    // backward loop
    c.dag = s->dag;
    c.narcs = g->arcs;
    const int mode = srv_mode(g->out);
    if (s->any_c) {
        // counting product of the pairs whose forward loop ended; their first
        // backward frontier joins the buffer the first backward round reads
        SHIP(hipMemcpyAsync(s->cmask, cm, ncg * 8, hipMemcpyHostToDevice, st));
        const size_t plane = (size_t)g->n * kWave;
        hipLaunchKernelGGL(k_srv_clear_flag, dim3(1), dim3(64), 0, st, s->flags + 1);
        hipLaunchKernelGGL(k_srv_pair_tau, dim3(nblocks((size_t)nc * plane, 256, 65536)), dim3(256), 0,
                           st, (const int32_t *)s->tdist, (uint32_t *)s->tau2, plane, s->ncg,
                           (const int32_t *)(s->cglists + 2 * ncg), nc, s->flags + 1);
        c.k = 0;
        c.ctr = s->ctr + ctr_slot(2, 0);
        c.clear_ctr = s->ctr + ctr_slot(2, 1);
        c.prev_ctr = nullptr;
        c.abits_n = s->abb[s->cur_b];
        c.fbits_n = s->bb[s->cur_b];
        c.abits = s->abb[s->cur_b ^ 1];
        c.fbits = s->bb[s->cur_b ^ 1];
        c.colmask = s->colmask + 32 * ncg;           // round 0, counting block
        c.cmask = s->cmask;
        c.nwide = nc;
        c.cglist = s->cglists + 2 * ncg;
        const int grid = nblocks((size_t)c.ntasks * nc, kWavesPerBlock, 0x7fffffff);
        switch (mode) {
            case 0:
                hipLaunchKernelGGL((k_bwd_count_w<0, true, false>), dim3(grid), dim3(kBlock), 0, st, c);
                hipLaunchKernelGGL((k_bwd_count_w<0, true, true>), dim3(grid), dim3(kBlock), 0, st, c);
                break;
            case 1:
                hipLaunchKernelGGL((k_bwd_count_w<1, true, false>), dim3(grid), dim3(kBlock), 0, st, c);
                hipLaunchKernelGGL((k_bwd_count_w<1, true, true>), dim3(grid), dim3(kBlock), 0, st, c);
                break;
            default:
                hipLaunchKernelGGL((k_bwd_count_w<2, true, false>), dim3(grid), dim3(kBlock), 0, st, c);
                hipLaunchKernelGGL((k_bwd_count_w<2, true, true>), dim3(grid), dim3(kBlock), 0, st, c);
                break;
        }
        // hub rows: the partial counts merged per group of the counted pairs
        BwdArgs m = c;
        m.ncg = ncgc;
        m.cglist = s->cglists + 3 * ncg;
        const int mgrid = nblocks((size_t)m.nhubs * ncgc, kWavesPerBlock, 0x7fffffff);
        hipLaunchKernelGGL(k_bwd_count_merge<true>, dim3(mgrid), dim3(kBlock), 0, st, m);
    }
    // R rounds of one forward product (every pair with a forward column) and
    // one backward product (every pair with a backward or just-counted
    // column).  A product whose predecessor in this step produced nothing for
    // any listed pair skips itself on the device (live_prev); a pair whose
    // loop ends within the step only runs products that find nothing for it.
    for (int r = 0; r < R; r++) {
        if (s->any_f) {
            const int b = s->cur_f;
            FwdArgs a{};
            a.tasks = g->plan_in.tasks;
            a.hubs = g->plan_in.hubs;
            a.ntasks = g->plan_in.ntasks;
            a.nhubs = g->plan_in.nhubs;
            a.nslots = g->plan_in.nslots;
            a.ncg = nf * kWide;
            a.ncg_all = s->ncg;
            a.nwide = nf;
            a.nwide_all = s->npair;
            a.cglist = s->cglists;
            a.n = g->n;
            a.j = ++s->kfwd;
            a.nwords = nw;
            a.mb = g->mb;
            a.rp = g->in.rp;
            a.arcs = srv_arc_src(g->in);
            a.abits = s->abf[b];
            a.ftup = s->ftup[b];
            a.fsig = s->fsig[b];
            a.tdist = s->tdist;
            a.tsig = s->tsig;
            a.abits_n = s->abf[b ^ 1];
            a.ftup_n = s->ftup[b ^ 1];
            a.fsig_n = s->fsig[b ^ 1];
            a.pd = s->pd;
            a.pm = s->pm;
            a.ctr = s->ctr + ctr_slot(0, r);
            a.prev_ctr = r > 0 ? s->ctr + ctr_slot(0, r - 1) : nullptr;
            a.flags = s->flags;
            a.clear_bits = s->abf[b];
            a.clear_ctr = s->ctr + ctr_slot(0, r + 1);
            a.colmask = s->colmask + (size_t)r * cmw;
            const int grid = nblocks((size_t)a.ntasks * nf, kWavesPerBlock, 0x7fffffff);
            switch (srv_mode(g->in)) {
                case 0: hipLaunchKernelGGL((k_fwd_pull_w<0, kWide, true>), dim3(grid), dim3(kBlock), 0, st, a); break;
                case 1: hipLaunchKernelGGL((k_fwd_pull_w<1, kWide, true>), dim3(grid), dim3(kBlock), 0, st, a); break;
                default: hipLaunchKernelGGL((k_fwd_pull_w<2, kWide, true>), dim3(grid), dim3(kBlock), 0, st, a); break;
            }
            const int mgrid = std::max(nblocks((size_t)a.nhubs * nf, kWavesPerBlock, 0x7fffffff),
                                       nblocks((size_t)nw, kBlock, 1024));
            hipLaunchKernelGGL((k_fwd_merge_w<kWide, true>), dim3(mgrid), dim3(kBlock), 0, st, a);
            s->cur_f ^= 1;
        }
        if (s->any_b) {
            // reads cur_b, writes the other
            const int b = s->cur_b;
            c.k = ++s->kbwd;
            c.ctr = s->ctr + ctr_slot(1, r);
            c.prev_ctr = r > 0 ? s->ctr + ctr_slot(1, r - 1) : nullptr;
            c.clear_ctr = s->ctr + ctr_slot(1, r + 1);
            c.abits = s->abb[b];
            c.fbits = s->bb[b];
            c.abits_n = s->abb[b ^ 1];
            c.fbits_n = s->bb[b ^ 1];
            c.clear_bits = s->abb[b];
            c.colmask = s->colmask + (size_t)r * cmw + 2 * 32 * ncg;
            c.cmask = nullptr;
            c.nwide = nbk;
            c.cglist = s->cglists + ncg;
            const int grid = nblocks((size_t)c.ntasks * nbk, kWavesPerBlock, 0x7fffffff);
            switch (mode) {
                case 0: hipLaunchKernelGGL((k_bwd_pull_w<0, true>), dim3(grid), dim3(kBlock), 0, st, c); break;
                case 1: hipLaunchKernelGGL((k_bwd_pull_w<1, true>), dim3(grid), dim3(kBlock), 0, st, c); break;
                default: hipLaunchKernelGGL((k_bwd_pull_w<2, true>), dim3(grid), dim3(kBlock), 0, st, c); break;
            }
            const int mgrid = std::max(nblocks((size_t)c.nhubs * nbk, kWavesPerBlock, 0x7fffffff),
                                       nblocks((size_t)nw, kBlock, 1024));
            hipLaunchKernelGGL(k_bwd_merge_w<true>, dim3(mgrid), dim3(kBlock), 0, st, c);
            s->cur_b ^= 1;
        }
    }
    SHIP(hipGetLastError());
    // the counting product's columns (round 0) and the last round's products
    SHIP(hipMemcpyAsync(s->h_colmask, s->colmask, cmw * 8, hipMemcpyDeviceToHost, st));
    SHIP(hipMemcpyAsync(s->h_colmask + cmw, s->colmask + (size_t)(R - 1) * cmw, cmw * 8,
                        hipMemcpyDeviceToHost, st));
    SHIP(hipMemcpyAsync(s->h_flags, s->flags, 4, hipMemcpyDeviceToHost, st));
    SHIP(hipEventRecord(s->done_ev, st));
    s->launched = true;
    if (prev >= 0) (void)hipSetDevice(prev);
    return MFBC_OK;
}

int mfbc_server_set_rounds(mfbc_server *s, int32_t rounds) {
    if (!s) return sfail(MFBC_EINVAL, "NULL server");
    if (rounds < 0 || rounds > kMaxRounds)
        return sfail(MFBC_EINVAL, "rounds must be in [0, " + std::to_string(kMaxRounds) + "]");
    if (s->launched) return sfail(MFBC_EINVAL, "a step is in flight");
    s->rounds = rounds;
    return MFBC_OK;
}

int mfbc_server_step_query(mfbc_server *s) {
    if (!s) return sfail(MFBC_EINVAL, "NULL server");
    if (!s->launched) return 1;
    const hipError_t e = hipEventQuery(s->done_ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return sfail(MFBC_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

int mfbc_server_step_finish(mfbc_server *s, int32_t *h_done, int32_t *h_ndone, void *hip_stream) {
    if (!s || !h_done || !h_ndone) return sfail(MFBC_EINVAL, "NULL argument");
    if (!s->launched) return sfail(MFBC_EINVAL, "no step in flight");
    SHIP(hipStreamSynchronize((hipStream_t)hip_stream));
    s->launched = false;
    if (s->h_flags[0])
        return sfail(MFBC_EOVERFLOW, "a shortest-path count overflowed binary64; the results of "
                                     "the columns in flight are invalid");
    const size_t ncg = (size_t)s->ncg;
    const size_t cmw = 3 * 32 * ncg;
    const unsigned long long *last = s->h_colmask + cmw;   // the step's last round
    std::vector<uint64_t> mf(ncg, 0), mc(ncg, 0), mb(ncg, 0);
    for (size_t k = 0; k < 32; k++)
        for (size_t c = 0; c < ncg; c++) {
            mf[c] |= last[k * ncg + c];
            mc[c] |= s->h_colmask[32 * ncg + k * ncg + c];
            mb[c] |= last[64 * ncg + k * ncg + c];
        }
    int nd = 0;
    for (int c = 0; c < s->width; c++) {
        // frontiers only shrink to empty: a pair of groups leaves the forward
        // loop when none of its lanes produced in the last round, a column its
        // backward loop when it produced nothing in the last round
        const size_t g0 = (size_t)(c / (kWide * kWave)) * kWide;
        const bool grp_f = mf[g0] != 0ull || (g0 + 1 < ncg && mf[g0 + 1] != 0ull);
        const bool bit_c = (mc[(size_t)(c / 64)] >> (c % 64)) & 1ull;
        const bool bit_b = (mb[(size_t)(c / 64)] >> (c % 64)) & 1ull;
        uint8_t &p = s->phase[(size_t)c];
        if (s->ran_f[(size_t)c] && p == kFwd && !grp_f) p = kCnt;
        else if (s->ran_c[(size_t)c] && p == kCnt) p = bit_c && bit_b ? kBwd : kDone;
        else if (s->ran_b[(size_t)c] && p == kBwd && !bit_b) p = kDone;
        if (p == kDone && (s->ran_b[(size_t)c] || s->ran_c[(size_t)c])) h_done[nd++] = c;
    }
    *h_ndone = nd;
    return MFBC_OK;
}

static int harvest_common(mfbc_server *s, const int32_t *h_columns, int32_t count) {
    for (int i = 0; i < count; i++) {
        const int c = h_columns[i];
        if (c < 0 || c >= s->width || s->phase[(size_t)c] != kDone)
            return sfail(MFBC_EINVAL, "column " + std::to_string(c) + " is not finished");
    }
    return MFBC_OK;
}

static void release(mfbc_server *s, const int32_t *h_columns, int32_t count) {
    for (int i = 0; i < count; i++) {
        s->phase[(size_t)h_columns[i]] = kFree;
        s->h_src[(size_t)h_columns[i]] = -1;
    }
}

int mfbc_server_harvest_bc(mfbc_server *s, const int32_t *h_columns, int32_t count,
                           double *const *d_dest, void *hip_stream) {
    if (!s || (count > 0 && (!h_columns || !d_dest))) return sfail(MFBC_EINVAL, "NULL argument");
    if (count <= 0) return MFBC_OK;
    int rc = harvest_common(s, h_columns, count);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const int ncg = s->ncg;
    // entries grouped by column group, each group's in list order
    std::vector<int32_t> gofs((size_t)ncg + 1, 0);
    for (int i = 0; i < count; i++) gofs[(size_t)(h_columns[i] / kWave) + 1]++;
    for (int g = 0; g < ncg; g++) gofs[(size_t)g + 1] += gofs[(size_t)g];
    std::vector<int32_t> pos(gofs.begin(), gofs.end() - 1);
    const size_t o_ptr = 0, o_col = (size_t)count * 8, o_gofs = o_col + (size_t)count * 4;
    const size_t bytes = o_gofs + ((size_t)ncg + 1) * 4;
    if ((rc = stage(s, bytes + 256))) return rc;
    std::vector<char> h(bytes, 0);
    double **hp = (double **)(h.data() + o_ptr);
    int32_t *hc = (int32_t *)(h.data() + o_col);
    for (int i = 0; i < count; i++) {
        const int k = pos[(size_t)(h_columns[i] / kWave)]++;
        hp[k] = d_dest[i];
        hc[k] = h_columns[i];
    }
    memcpy(h.data() + o_gofs, gofs.data(), ((size_t)ncg + 1) * 4);
    SHIP(hipMemcpyAsync(s->meta, h.data(), bytes, hipMemcpyHostToDevice, st));
    const int n = s->g->n;
    hipLaunchKernelGGL(k_srv_harvest_bc, dim3((n + 63) / 64), dim3(256), 0, st, n, ncg,
                       (const int32_t *)(s->meta + o_col), (const int32_t *)(s->meta + o_gofs),
                       (const int32_t *)s->src, (double *const *)(s->meta + o_ptr),
                       (const int32_t *)s->tdist, (const double *)s->tsig, (const double *)s->zeta,
                       (const int32_t *)s->g->perm);
    SHIP(hipGetLastError());
    SHIP(hipStreamSynchronize(st));
    release(s, h_columns, count);
    return MFBC_OK;
}

int mfbc_server_harvest_dep(mfbc_server *s, const int32_t *h_columns, int32_t count,
                            const int32_t *d_targets, int32_t ntargets, double *const *d_out,
                            void *hip_stream) {
    if (!s || (count > 0 && (!h_columns || !d_out)) || ntargets < 0 || (ntargets > 0 && !d_targets))
        return sfail(MFBC_EINVAL, "bad argument");
    if (count <= 0) return MFBC_OK;
    int rc = harvest_common(s, h_columns, count);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<int32_t> ht((size_t)ntargets);
    if (ntargets) {
        SHIP(hipMemcpyAsync(ht.data(), d_targets, (size_t)ntargets * 4, hipMemcpyDeviceToHost, st));
        SHIP(hipStreamSynchronize(st));
        for (int32_t t : ht)
            if (t < 0 || t >= s->g->n) return sfail(MFBC_EINVAL, "target out of range");
    }
    if ((rc = stage(s, (size_t)count * 12 + 256))) return rc;
    std::vector<char> h((size_t)count * 12 + 256, 0);
    const size_t o_ptr = 0, o_col = (size_t)count * 8;
    memcpy(h.data() + o_ptr, d_out, (size_t)count * 8);
    memcpy(h.data() + o_col, h_columns, (size_t)count * 4);
    SHIP(hipMemcpyAsync(s->meta, h.data(), (size_t)count * 12, hipMemcpyHostToDevice, st));
    if (ntargets)
        hipLaunchKernelGGL(k_srv_harvest_dep, dim3(nblocks((size_t)count * ntargets, 256)), dim3(256),
                           0, st, s->g->n, (const int32_t *)(s->meta + o_col), count,
                           (const int32_t *)s->src, d_targets, ntargets,
                           (double *const *)(s->meta + o_ptr), (const int32_t *)s->tdist,
                           (const double *)s->tsig, (const double *)s->zeta,
                           (const int32_t *)s->g->perm);
    SHIP(hipGetLastError());
    SHIP(hipStreamSynchronize(st));
    release(s, h_columns, count);
    return MFBC_OK;
}

}  // extern "C"
