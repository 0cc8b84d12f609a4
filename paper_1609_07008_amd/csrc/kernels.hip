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
//    The counting product also stores the shortest-path DAG: for every arc,
//    the lane mask of the sources for which the arc is on a shortest path.
//  * Backward product (Algorithm 2, loop): for each pending (s, x), the sum of
//    the frontier values q(s,y) = zeta(s,y) + 1/sigma(s,y) over frontier
//    successors y, and the number of them, which is taken off x's counter;
//    x joins the next frontier when its counter reaches zero.  An arc x -> y
//    counts in lane s iff y's frontier lane mask and the arc's DAG mask both
//    have bit s.
//  * lambda (Algorithm 3): delta(s,x) = zeta(s,x) * sigma(s,x) is added to a
//    per-(column group, vertex) partial when (s,x) completes; the source's
//    own entry is excluded (sigma(s,t,s) = 0 in Section 2.4).
//
// Activity filter: a one-bit-per-vertex bitmap per column group (any of its
// 64 columns active; n/8 bytes, resident in L2) is checked per arc first.
// The forward product then reads the neighbour's whole 256-B tuple row
// (absent lanes hold a sentinel); the backward product reads the 64-bit
// lane masks and gathers q only for the lanes that count.  Batches of two
// or more column groups run the forward product (and on weighted graphs the
// backward products) on pairs of groups: one 8-byte (16-byte) gather per
// lane and one bitmap test per arc serve both groups (products.h).
#include "products.h"

namespace mfbc {
namespace {
// ===================================================================== setup / io
// In every kernel here `perm` (nullable) maps a caller vertex id to the
// device numbering; the products themselves only see device ids.
__device__ __forceinline__ int dev_id(const int32_t *perm, int v) { return perm ? perm[v] : v; }

__global__ void k_set_sources(int32_t *src, int total, int nb, const int32_t *in,
                              const int32_t *perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) src[i] = i < nb ? dev_id(perm, in[i]) : -1;
}

// Sources of a batch laid out by request (mfbc_bc_requests): group slot cg
// holds sp.count[cg] consecutive sources from in[sp.first[cg]] on and
// padding (-1) after them.
__global__ void k_set_sources_spans(int32_t *src, int ncg, const int32_t *in, GroupSpans sp,
                                    const int32_t *perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncg * kWave) return;
    const int cg = i / kWave, l = i % kWave;
    src[i] = l < sp.count[cg] ? dev_id(perm, in[sp.first[cg] + l]) : -1;
}

// *bad = 1 if some listed source is outside [0, n) (bad must start at 0).
__global__ void k_check_sources(const int32_t *src, int64_t count, int n, int32_t *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        if (src[i] < 0 || src[i] >= n) *bad = 1;
}

// Zero `count` 32-bit words (a kernel rather than a memset node, so that a
// stream capture records no memset).
__global__ void k_zero_u32(uint32_t *p, size_t count) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0u;
}

// T = (INF, 0) everywhere, both frontier bitmaps cleared, counters zeroed.
__global__ void k_fwd_fill(int32_t *tdist, double *tsig, size_t total, uint32_t *ab0, uint32_t *ab1,
                           size_t nab, unsigned long long *ctr, int nctr, int32_t *flags) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    // sigma is read only where tau is finite (ties in the forward product,
    // leaves and finishes in the backward, exports masked by tau), so only
    // tau is reset
    for (size_t i = t0; i < total; i += stride) tdist[i] = kInf;
    (void)tsig;
    for (size_t i = t0; i < nab; i += stride) {
        ab0[i] = 0u;
        ab1[i] = 0u;
    }
    for (size_t i = t0; i < (size_t)nctr; i += stride) ctr[i] = 0ull;
    if (t0 == 0) flags[0] = 0;
}

// Rows of the sources in the first frontier start with every lane absent.
__global__ void k_fwd_seed_rows(const int32_t *src, int nb, int n, uint32_t *ftup) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb || src[c] < 0) return;          // padding column
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
    if (v < 0) return;                           // padding column
    const int cg = c / kWave, lane = c % kWave;
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    tdist[idx] = 0;
    tsig[idx] = 1.0;
    ftup[idx] = 1u;                      // weight 0, multiplicity 1 inline
    atomicOr(abits + (size_t)cg * nwords + (v >> 5), 1u << (v & 31));
}

// The same for the wide layout (groups Wq .. Wq+W-1 interleaved per lane,
// one activity bitmap per wide group).
template <int W>
__global__ void k_fwd_seed_rows_w(const int32_t *src, int nb, int n, uint32_t *ftup) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb || src[c] < 0) return;          // padding column
    const size_t row = ((size_t)(c / (W * kWave)) * n + src[c]) * kWave * W;
    for (int l = 0; l < kWave * W; l++) ftup[row + l] = kSent;
}

template <int W>
__global__ void k_fwd_seed_w(const int32_t *src, int nb, int n, int nwords, int32_t *tdist,
                             double *tsig, uint32_t *ftup, uint32_t *abits) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int v = src[c];
    if (v < 0) return;                           // padding column
    const int cg = c / kWave, lane = c % kWave, q = cg / W;
    const size_t idx = ((size_t)cg * n + v) * kWave + lane;
    tdist[idx] = 0;
    tsig[idx] = 1.0;
    ftup[(((size_t)q * n + v) * kWave + lane) * W + (cg % W)] = 1u;
    atomicOr(abits + (size_t)q * nwords + (v >> 5), 1u << (v & 31));
}

__global__ void k_zero_f64(double *p, size_t total) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) p[i] = 0.0;
}

// bc[v] for caller vertex v (written in caller order, coalesced).
__global__ void k_lambda_reduce(const double *lam, int ncg, int n, double *bc,
                                const int32_t *perm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int d = dev_id(perm, v);
    double t = 0.0;
    for (int cg = 0; cg < ncg; cg++) t += lam[(size_t)cg * n + d];
    bc[v] = t;
}

// lambda parts of each group slot added to the sum of the request that owns
// the slot (mfbc_bc_requests), caller numbering; slots in ascending order,
// so a request with several slots is summed in a fixed order.
__global__ void k_lambda_add_groups(const double *lam, int ncg, int n, GroupOuts o,
                                    const int32_t *perm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int d = dev_id(perm, v);
    for (int cg = 0; cg < ncg; cg++)
        if (o.out[cg]) o.out[cg][v] += lam[(size_t)cg * n + d];
}

// The same over the workspaces of several lanes (fixed lane order).
struct LanePtrs {
    const double *lam[kMaxLanes];
};

__global__ void k_lambda_reduce_lanes(LanePtrs p, int nlanes, int ncg, int n, double *bc,
                                      const int32_t *perm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int d = dev_id(perm, v);
    double t = 0.0;
    for (int l = 0; l < nlanes; l++)
        for (int cg = 0; cg < ncg; cg++) t += p.lam[l][(size_t)cg * n + d];
    bc[v] = t;
}

// Tile transposes between [cg][v][64] tiles (device numbering) and
// source-major rows [s][v] (caller numbering), 64 x 64 per block through LDS
// (padded against bank conflicts).  A block covers 64 consecutive caller
// vertices: the row side stays coalesced, the tile side moves whole 256-B
// tile rows.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tiles_to_rows(const T *tiles, T *rows, int n, int nb,
                                                          const int32_t *perm) {
    __shared__ T sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) sh[r][c] = tiles[((size_t)cg * n + dev_id(perm, v)) * 64 + c];
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        if (s < nb && v < n) rows[(size_t)s * n + v] = sh[c][r];
    }
}

// sigma tiles to rows, 0 where tau is infinite (sigma is not reset there).
__global__ __launch_bounds__(kBlock) void k_sigma_rows(const double *tsig, const int32_t *tdist,
                                                       double *rows, int n, int nb,
                                                       const int32_t *perm) {
    __shared__ double sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) {
            const size_t idx = ((size_t)cg * n + dev_id(perm, v)) * 64 + c;
            sh[r][c] = tdist[idx] != kInf ? tsig[idx] : 0.0;
        }
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        if (s < nb && v < n) rows[(size_t)s * n + v] = sh[c][r];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rows_to_tiles(const T *rows, T *tiles, int n, int nb,
                                                          T pad, const int32_t *perm) {
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
        if (v < n) tiles[((size_t)cg * n + dev_id(perm, v)) * 64 + c] = sh[r][c];
    }
}

// delta(s, v) = zeta(s, v) * sigma(s, v), 0 at the source and where unreachable.
__global__ __launch_bounds__(kBlock) void k_delta_rows(const double *zeta, const double *tsig,
                                                       const int32_t *tdist, const int32_t *src,
                                                       double *rows, int n, int nb,
                                                       const int32_t *perm) {
    __shared__ double sh[64][65];
    const int cg = blockIdx.y, v0 = blockIdx.x * 64;
    const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    for (int r = r0; r < 64; r += 4) {
        const int v = v0 + r;
        if (v < n) {
            const int d = dev_id(perm, v);
            const size_t idx = ((size_t)cg * n + d) * 64 + c;
            const bool ok = tdist[idx] != kInf && src[cg * 64 + c] != d;
            sh[r][c] = ok ? zeta[idx] * tsig[idx] : 0.0;
        }
    }
    __syncthreads();
    for (int r = r0; r < 64; r += 4) {
        const int s = cg * 64 + r, v = v0 + c;
        if (s < nb && v < n) rows[(size_t)s * n + v] = sh[c][r];
    }
}

// The counting product of a batch of two or more groups reads tau of each
// pair of groups interleaved per lane in 16 bits a group: tau2[q][v][lane] =
// (tau of group 2q, tau of group 2q+1) at (v, lane), packed by pack_tau16; a
// padding group reads as unreachable.  *full (cleared before) is set when a
// finite tau does not fit.
__global__ void k_pair_tau(const int32_t *tdist, uint32_t *tau2, size_t plane, int ncg, int npairs,
                           int32_t *full) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t total = (size_t)npairs * plane;
    bool big = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const size_t q = i / plane, r = i - q * plane;
        const int x = tdist[2 * q * plane + r];
        const int y = (int)(2 * q + 1) < ncg ? tdist[(2 * q + 1) * plane + r] : kInf;
        big |= tau16_big(x) || tau16_big(y);
        tau2[i] = pack_tau16(x, y);
    }
    if (big) *full = 1;
}

// Trace of forward frontier F_j: one wave per (source column c, 64 caller
// vertices); lane v tests the vertex's activity bit and its tuple in the
// frontier buffers, the wave's ballot is the bitmap word.  The out-degrees
// of the members are summed into *relax (the relaxations of the next
// product: each frontier entry is combined once along each of its arcs).
__global__ __launch_bounds__(kBlock) void k_trace_fwd(const uint32_t *abits, const uint32_t *ftup,
                                                      int n, int nwords, int nb, int wide,
                                                      const int32_t *perm, const int64_t *rp_out,
                                                      uint64_t *rows, int words64,
                                                      unsigned long long *relax) {
    const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & (kWave - 1);
    const size_t c = wave / (size_t)words64;
    const int wv = (int)(wave - c * (size_t)words64);
    bool member = false;
    unsigned long long r = 0;
    const int v = wv * kWave + lane;
    if (c < (size_t)nb && v < n) {
        const int d = dev_id(perm, v);
        const int cg = (int)(c / kWave), l = (int)(c % kWave);
        const int plane = wide ? cg >> 1 : cg;
        if ((abits[(size_t)plane * nwords + (d >> 5)] >> (d & 31)) & 1u) {
            const size_t idx = wide ? ((((size_t)plane * n + d) * kWave + l) * 2 + (cg & 1))
                                    : (((size_t)cg * n + d) * kWave + l);
            member = ftup[idx] != kSent;
            if (member) r = (unsigned long long)(rp_out[d + 1] - rp_out[d]);
        }
    }
    const uint64_t word = ballot(member);
    if (c < (size_t)nb && lane == 0 && rows) rows[c * (size_t)words64 + wv] = word;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) r += __shfl_xor(r, off, kWave);
    if (lane == 0 && r) atomicAdd(relax, r);
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

// Batches of two or more column groups run the forward product on pairs of
// them (the workspace holds an even number of groups); a single group runs
// alone.
static int fwd_wide_groups(int ncg) { return ncg >= 2 ? (ncg + kWide - 1) / kWide : 0; }

static FwdArgs fwd_args(mfbc_graph *g, int ncg, int j) {
    Workspace &ws = g->ws;
    const int b = (j - 1) & 1;  // buffer holding F_{j-1}
    FwdArgs a{};
    a.tasks = g->plan_in.tasks;
    a.hubs = g->plan_in.hubs;
    a.ntasks = g->plan_in.ntasks;
    a.nhubs = g->plan_in.nhubs;
    a.nslots = g->plan_in.nslots;
    a.ncg = ncg;
    a.ncg_all = ncg;
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
    a.prev_ctr = j > 1 ? ws.counters + (size_t)((j - 1) % kCounterRing) * 4 * kCounterSlots : nullptr;
    a.flags = ws.flags;
    a.clear_bits = ws.abits[b];
    a.clear_ctr = ws.counters + (size_t)((j + 1) % kCounterRing) * 4 * kCounterSlots;
    a.nwide = fwd_wide_groups(ncg);
    a.nwide_all = a.nwide;
    return a;
}

void launch_check_sources(const int32_t *d_sources, int64_t count, int n, int32_t *d_bad,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (uint32_t *)d_bad, (size_t)1);
    if (count > 0)
        hipLaunchKernelGGL(k_check_sources, dim3(blocks_for((size_t)count, 256, 4096)), dim3(256), 0, s,
                           d_sources, count, n, d_bad);
}

void launch_set_sources(mfbc_graph *g, int ncg, int nb, const int32_t *d_sources, hipStream_t s) {
    const int total = ncg * kWave;
    hipLaunchKernelGGL(k_set_sources, dim3(blocks_for(total, 256)), dim3(256), 0, s, g->ws.src,
                       total, nb, d_sources, (const int32_t *)g->perm);
}

void launch_fwd_init(mfbc_graph *g, int ncg, int nb, hipStream_t s) {
    Workspace &ws = g->ws;
    const size_t total = (size_t)ncg * g->n * kWave;
    const int nwords = (g->n + 31) / 32;
    hipLaunchKernelGGL(k_fwd_fill, dim3(blocks_for(total, 256, 65536)), dim3(256), 0, s, ws.tdist,
                       ws.tsig, total, ws.abits[0], ws.abits[1], (size_t)ncg * nwords,
                       ws.counters, kCounterRing * 4 * kCounterSlots, ws.flags);
    if (fwd_wide_groups(ncg)) {
        uint32_t *ft = (uint32_t *)ws.fdist[0];
        hipLaunchKernelGGL(k_fwd_seed_rows_w<kWide>, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src,
                           nb, g->n, ft);
        hipLaunchKernelGGL(k_fwd_seed_w<kWide>, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src, nb,
                           g->n, nwords, ws.tdist, ws.tsig, ft, ws.abits[0]);
        return;
    }
    hipLaunchKernelGGL(k_fwd_seed_rows, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src, nb,
                       g->n, (uint32_t *)ws.fdist[0]);
    hipLaunchKernelGGL(k_fwd_seed, dim3(blocks_for(nb, 256)), dim3(256), 0, s, ws.src, nb, g->n,
                       nwords, ws.tdist, ws.tsig, (uint32_t *)ws.fdist[0], ws.abits[0]);
}

void launch_fwd_product(mfbc_graph *g, int ncg, int j, hipStream_t s, hipEvent_t *ev) {
    FwdArgs a = fwd_args(g, ncg, j);
    if (a.nwide) {
        if (ev) (void)hipEventRecord(ev[0], s);
        const int grid = blocks_for((size_t)a.ntasks * a.nwide, kWavesPerBlock, 0x7fffffff);
        switch (arc_mode(g->in)) {
            case 0: hipLaunchKernelGGL((k_fwd_pull_w<0, kWide, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_fwd_pull_w<1, kWide, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            default: hipLaunchKernelGGL((k_fwd_pull_w<2, kWide, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        }
        if (ev) (void)hipEventRecord(ev[1], s);
        int mgrid = blocks_for((size_t)a.nhubs * a.nwide, kWavesPerBlock, 0x7fffffff);
        const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
        if (cgrid > mgrid) mgrid = cgrid;
        hipLaunchKernelGGL((k_fwd_merge_w<kWide, false>), dim3(mgrid), dim3(kBlock), 0, s, a);
        if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
        return;
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    const size_t waves = (size_t)a.ntasks * ncg;
    const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
    switch (arc_mode(g->in)) {
        case 0: hipLaunchKernelGGL((k_fwd_pull<0, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_fwd_pull<1, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_fwd_pull<2, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
    }
    if (ev) (void)hipEventRecord(ev[1], s);
    const size_t mw = (size_t)a.nhubs * ncg;
    int mgrid = blocks_for(mw, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_fwd_merge<false>, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
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
    a.ncg_all = ncg;
    a.n = g->n;
    a.k = k;
    a.rp = g->out.rp;
    a.arcs = arc_src(g->out);
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
    a.step = g->trace_step ? ws.fdist[1] : nullptr;   // frontier indices only when traced
    a.lam = ws.lam;
    a.dag = ws.dag;
    a.narcs = g->arcs;
    a.pd = ws.pd;
    a.pm = ws.pm;
    a.ctr = ws.counters + (size_t)(k % kCounterRing) * 4 * kCounterSlots;
    a.prev_ctr = k > 0 ? ws.counters + (size_t)((k - 1) % kCounterRing) * 4 * kCounterSlots : nullptr;
    a.tau2 = (const uint32_t *)ws.tau2;
    a.tau_full = ws.flags + 1;
    a.nwords = (g->n + 31) / 32;
    a.clear_bits = ws.abits[b];
    a.clear_ctr = ws.counters + (size_t)((k + 1) % kCounterRing) * 4 * kCounterSlots;
    // on weighted graphs the backward products run on pairs of groups like
    // the forward one (one pass over the arcs and one lane-mask gather serve
    // both).  Unweighted graphs tie often, their DAG masks are dense and the
    // per-arc value gathers dominate: there the pair form, at two arcs per
    // round and five waves per SIMD, measured slower (rmat16: 15.9 against
    // 13.4 ms per step) and one group per wave is kept.
    a.nwide = arc_mode(g->out) != 0 ? fwd_wide_groups(ncg) : 0;
    a.nwide_all = a.nwide;
    return a;
}

hipError_t launch_bwd_count(mfbc_graph *g, int ncg, hipStream_t s, hipEvent_t *ev) {
    Workspace &ws = g->ws;
    // the counting product writes B_0 into buffer 0: clear its bitmap and
    // this product's counters first
    const int nwords = (g->n + 31) / 32;
    const size_t nab = (size_t)nwords * ncg;
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nab, 256, 4096)), dim3(256), 0, s, ws.abits[0], nab);
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nab, 256, 4096)), dim3(256), 0, s, ws.abits[1], nab);
    const size_t nctr = (size_t)kCounterRing * 4 * kCounterSlots * 2;   // u64 counters as u32 words
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(nctr, 256)), dim3(256), 0, s,
                       (uint32_t *)ws.counters, nctr);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, (uint32_t *)ws.flags + 1, (size_t)1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BwdArgs a = bwd_args(g, ncg, 0);
    if (ev) (void)hipEventRecord(ev[0], s);
    if (ncg >= 2) {
        // pairs of groups: tau interleaved per pair, then one wave per (pair, task)
        const int npairs = (ncg + 1) / 2;
        const size_t plane = (size_t)g->n * kWave;
        hipLaunchKernelGGL(k_pair_tau, dim3(blocks_for((size_t)npairs * plane, 256, 65536)), dim3(256),
                           0, s, (const int32_t *)ws.tdist, (uint32_t *)ws.tau2, plane, ncg, npairs, ws.flags + 1);
        const int grid = blocks_for((size_t)a.ntasks * npairs, kWavesPerBlock, 0x7fffffff);
        switch (arc_mode(g->out)) {
            case 0:
                hipLaunchKernelGGL((k_bwd_count_w<0, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
                hipLaunchKernelGGL((k_bwd_count_w<0, false, true>), dim3(grid), dim3(kBlock), 0, s, a);
                break;
            case 1:
                hipLaunchKernelGGL((k_bwd_count_w<1, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
                hipLaunchKernelGGL((k_bwd_count_w<1, false, true>), dim3(grid), dim3(kBlock), 0, s, a);
                break;
            default:
                hipLaunchKernelGGL((k_bwd_count_w<2, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
                hipLaunchKernelGGL((k_bwd_count_w<2, false, true>), dim3(grid), dim3(kBlock), 0, s, a);
                break;
        }
    } else {
        const size_t waves = (size_t)a.ntasks * ncg;
        const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
        switch (arc_mode(g->out)) {
            case 0: hipLaunchKernelGGL((k_bwd_count<0, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_bwd_count<1, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            default: hipLaunchKernelGGL((k_bwd_count<2, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        }
    }
    if (ev) (void)hipEventRecord(ev[1], s);
    int mgrid = blocks_for((size_t)a.nhubs * ncg, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_bwd_count_merge<false>, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
    return hipGetLastError();
}

void launch_bwd_product(mfbc_graph *g, int ncg, int k, hipStream_t s, hipEvent_t *ev) {
    BwdArgs a = bwd_args(g, ncg, k);
    if (a.nwide) {
        if (ev) (void)hipEventRecord(ev[0], s);
        const int grid = blocks_for((size_t)a.ntasks * a.nwide, kWavesPerBlock, 0x7fffffff);
        switch (arc_mode(g->out)) {
            case 0: hipLaunchKernelGGL((k_bwd_pull_w<0, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_bwd_pull_w<1, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
            default: hipLaunchKernelGGL((k_bwd_pull_w<2, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        }
        if (ev) (void)hipEventRecord(ev[1], s);
        int mgrid = blocks_for((size_t)a.nhubs * a.nwide, kWavesPerBlock, 0x7fffffff);
        const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
        if (cgrid > mgrid) mgrid = cgrid;
        hipLaunchKernelGGL(k_bwd_merge_w<false>, dim3(mgrid), dim3(kBlock), 0, s, a);
        if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
        return;
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    const size_t waves = (size_t)a.ntasks * ncg;
    const int grid = blocks_for(waves, kWavesPerBlock, 0x7fffffff);
    switch (arc_mode(g->out)) {
        case 0: hipLaunchKernelGGL((k_bwd_pull<0, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_bwd_pull<1, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_bwd_pull<2, false>), dim3(grid), dim3(kBlock), 0, s, a); break;
    }
    if (ev) (void)hipEventRecord(ev[1], s);
    int mgrid = blocks_for((size_t)a.nhubs * ncg, kWavesPerBlock, 0x7fffffff);
    const int cgrid = blocks_for((size_t)a.nwords, kBlock, 1024);
    if (cgrid > mgrid) mgrid = cgrid;
    hipLaunchKernelGGL(k_bwd_merge<false>, dim3(mgrid), dim3(kBlock), 0, s, a);
    if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
}

void launch_lambda_zero(mfbc_graph *g, int ncg, hipStream_t s) {
    const size_t total = (size_t)ncg * g->n;
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(total, 256, 65536)), dim3(256), 0, s, g->ws.lam,
                       total);
}

void launch_set_sources_spans(mfbc_graph *g, int ncg, const int32_t *d_sources,
                              const GroupSpans &sp, hipStream_t s) {
    hipLaunchKernelGGL(k_set_sources_spans, dim3(blocks_for(ncg * kWave, 256)), dim3(256), 0, s,
                       g->ws.src, ncg, d_sources, sp, (const int32_t *)g->perm);
}

void launch_lambda_add_groups(mfbc_graph *g, int ncg, const GroupOuts &o, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_add_groups, dim3(blocks_for(g->n, 256)), dim3(256), 0, s, g->ws.lam,
                       ncg, g->n, o, (const int32_t *)g->perm);
}

void launch_zero_f64(double *p, size_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(count, 256, 65536)), dim3(256), 0, s, p, count);
}

void launch_lambda_reduce(mfbc_graph *g, int ncg, double *d_bc, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_reduce, dim3(blocks_for(g->n, 256)), dim3(256), 0, s, g->ws.lam,
                       ncg, g->n, d_bc, (const int32_t *)g->perm);
}

void launch_lambda_reduce_lanes(mfbc_graph *const *lanes, int nlanes, int ncg, double *d_bc,
                                hipStream_t s) {
    LanePtrs p{};
    for (int l = 0; l < nlanes && l < kMaxLanes; l++) p.lam[l] = lanes[l]->ws.lam;
    const mfbc_graph *g = lanes[0];
    hipLaunchKernelGGL(k_lambda_reduce_lanes, dim3(blocks_for(g->n, 256)), dim3(256), 0, s, p, nlanes,
                       ncg, g->n, d_bc, (const int32_t *)g->perm);
}

void launch_export_forward(mfbc_graph *g, int ncg, int nb, int32_t *d_dist, double *d_sigma,
                           hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    const int32_t *perm = g->perm;
    hipLaunchKernelGGL(k_tiles_to_rows<int32_t>, grid, dim3(kBlock), 0, s, g->ws.tdist, d_dist,
                       g->n, nb, perm);
    hipLaunchKernelGGL(k_sigma_rows, grid, dim3(kBlock), 0, s, (const double *)g->ws.tsig,
                       (const int32_t *)g->ws.tdist, d_sigma, g->n, nb, perm);
}

void launch_trace_fwd(mfbc_graph *g, int ncg, int nb, int j, uint64_t *d_rows, hipStream_t s) {
    Workspace &ws = g->ws;
    const int b = j & 1;      // F_j sits in the buffers product j wrote (F_0: buffer 0)
    const int words64 = (g->n + 63) / 64;
    const size_t waves = (size_t)nb * words64;
    hipLaunchKernelGGL(k_trace_fwd, dim3(blocks_for(waves, kWavesPerBlock, 0x7fffffff)), dim3(kBlock),
                       0, s, (const uint32_t *)ws.abits[b], (const uint32_t *)ws.fdist[b], g->n,
                       (g->n + 31) / 32, nb, fwd_wide_groups(ncg) ? 1 : 0, (const int32_t *)g->perm,
                       (const int64_t *)g->out.rp, d_rows, words64, ws.trace_relax + j);
}

void launch_export_tiles_i32(mfbc_graph *g, int ncg, int nb, const int32_t *tiles, int32_t *d_rows,
                             hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    hipLaunchKernelGGL(k_tiles_to_rows<int32_t>, grid, dim3(kBlock), 0, s, tiles, d_rows, g->n, nb,
                       (const int32_t *)g->perm);
}

void launch_import_forward(mfbc_graph *g, int ncg, int nb, const int32_t *d_dist,
                           const double *d_sigma, hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    const int32_t *perm = g->perm;
    hipLaunchKernelGGL(k_rows_to_tiles<int32_t>, grid, dim3(kBlock), 0, s, d_dist, g->ws.tdist,
                       g->n, nb, (int32_t)kInf, perm);
    hipLaunchKernelGGL(k_rows_to_tiles<double>, grid, dim3(kBlock), 0, s, d_sigma, g->ws.tsig,
                       g->n, nb, 0.0, perm);
}

void launch_export_backward(mfbc_graph *g, int ncg, int nb, double *d_delta, int32_t *d_step,
                            hipStream_t s) {
    dim3 grid((g->n + 63) / 64, ncg);
    hipLaunchKernelGGL(k_delta_rows, grid, dim3(kBlock), 0, s, (const double *)g->ws.fsig[0],
                       (const double *)g->ws.tsig, (const int32_t *)g->ws.tdist,
                       (const int32_t *)g->ws.src, d_delta, g->n, nb, (const int32_t *)g->perm);
    if (d_step)
        hipLaunchKernelGGL(k_tiles_to_rows<int32_t>, grid, dim3(kBlock), 0, s,
                           (const int32_t *)g->ws.fdist[1], d_step, g->n, nb,
                           (const int32_t *)g->perm);
}

}  // namespace mfbc
