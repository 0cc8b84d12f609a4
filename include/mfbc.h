/*
 * mfbc.h -- C ABI of libmfbc: maximal frontier betweenness centrality (MFBC)
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Solomonik, Besta, Vella, Hoefler, "Scaling Betweenness Centrality
 * using Communication-Efficient Sparse Matrix Multiplication", SC17.
 *   - MFBF (Section 4.1, Algorithm 1): shortest distances and path counts of
 *     a batch of sources by repeated products of a frontier of multpaths
 *     (weight, multiplicity) with the adjacency matrix; the multpath monoid
 *     keeps the least weight and adds the multiplicities of ties; the next
 *     frontier keeps the entries no heavier than what is already known.
 *   - MFBr (Section 4.2, Algorithm 2): partial centrality factors
 *     zeta = delta / sigma by products of centpath frontiers (weight, partial
 *     centrality, counter) with the transposed adjacency, a vertex joining
 *     the frontier once all its shortest-path successors have reported.
 *   - MFBC (Section 4.3, Algorithm 3): lambda accumulated batch by batch.
 * Definitions (Section 2.4, Table 1): tau(s,v) distance, sigma(s,v) number
 * of shortest paths, delta(s,v) = sum_t sigma(s,t,v)/sigma(s,t) with
 * sigma(s,t,s) = sigma(s,t,t) = 0, lambda(v) = sum_s delta(s,v) over ordered
 * pairs, no halving or normalisation.
 *
 * Conventions shared by every call
 *   - Status: every int-returning call returns MFBC_OK (0) or a negative
 *     MFBC_E* code; mfbc_last_error() then describes the failure (a
 *     thread-local string, valid until the next call on that thread).
 *     Arguments are validated before any device work; on an error no output
 *     has been written.
 *   - Device pointers ("d_") are caller-owned device memory of the current
 *     HIP device (for example torch tensors); host pointers ("h_") are plain
 *     host memory.  The library owns only the graph and its workspace.
 *   - Workspace: a batch of nb sources (ceil(nb/64) groups of 64 columns,
 *     rounded up to an even count) takes about 37 B per (column, vertex) --
 *     T and two frontier buffers, which the backward state reuses -- plus
 *     8 B per (group of 64 columns, arc) for the shortest-path DAG that the
 *     counting product stores for the backward products (1 GiB at 2^25 arcs
 *     and 256 columns).  It grows to the largest batch seen and is freed
 *     with the graph; ENOMEM if it does not fit.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Calls are
 *     ordered on that stream and return after their outputs are complete
 *     (they synchronise on the stream to read frontier sizes: products are
 *     enqueued eight at a time and their frontier sizes read back once per
 *     eight; a product that follows one which produced nothing returns on
 *     the device without work).
 *   - Source-major outputs are row-major [nb][n]: entry (s, v) at s*n + v,
 *     where s indexes the listed sources.
 *   - A graph handle may be used by one thread at a time.
 */
#ifndef MFBC_H
#define MFBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFBC_INF_DIST 0x7fffffff /* distance of an unreachable vertex */

enum mfbc_status {
    MFBC_OK = 0,
    MFBC_EINVAL = -1,    /* malformed argument, graph or source          */
    MFBC_ENOMEM = -2,    /* device or host allocation failed              */
    MFBC_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed    */
    MFBC_EOVERFLOW = -4  /* distances could exceed int32, or a path count */
                         /* overflowed binary64                           */
};

enum mfbc_flags {
    MFBC_UNDIRECTED = 1, /* symmetric CSR required and checked            */
    MFBC_DIRECTED = 2,   /* CSR lists out-arcs; distances follow arcs     */
    MFBC_KEEP_ORDER = 4  /* or-ed in: store vertices in the caller's order */
};

typedef struct mfbc_graph mfbc_graph;

/*
 * mfbc_load_graph -- copy a graph to the device (the adjacency matrix A of
 * Section 2.1: A(u,v) = weight of arc u->v, absent arcs are infinite).
 *   n        vertices, 1 <= n < 2^31 - 1.
 *   n_arcs   number of arcs (2m for an undirected graph with m edges).
 *   h_row_ptr[n+1], h_col_idx[n_arcs]: host CSR of out-arcs; row_ptr[0] = 0,
 *            non-decreasing, row_ptr[n] = n_arcs; each row's columns strictly
 *            increasing (no duplicate arcs), in [0,n), no self-loops.
 *   h_weight[n_arcs]: host integer weights >= 1, or NULL (every weight 1).
 *            Zero or negative weights are rejected (zero-weight cycles would
 *            give infinitely many shortest walks).
 *   flags    MFBC_UNDIRECTED (the CSR must be symmetric with equal weights on
 *            both arcs) or MFBC_DIRECTED, optionally or-ed with
 *            MFBC_KEEP_ORDER.  Without it the device copy numbers vertices
 *            by descending degree (ties in the caller's order), which packs
 *            the frontier rows gathered most often into fewer memory pages;
 *            the renumbering is internal: every entry point takes and
 *            returns the caller's vertex ids and per-vertex arrays in the
 *            caller's order, and results equal those of MFBC_KEEP_ORDER up
 *            to the summation order of floating-point sums.
 *   out      receives the handle.
 * Errors: EINVAL (malformed CSR, weight <= 0, asymmetric undirected input),
 * EOVERFLOW (n * max weight >= 2^31 - 1), ENOMEM, EDEVICE.
 */
int mfbc_load_graph(int32_t n, int64_t n_arcs, const int64_t *h_row_ptr,
                    const int32_t *h_col_idx, const int32_t *h_weight,
                    uint32_t flags, void *hip_stream, mfbc_graph **out);

/* Release a graph and its device workspace (NULL is accepted).
 * Errors: EINVAL while servers created on the graph (mfbc_server_create) are
 * live; the graph is then left as it was, and is freed by a call made after
 * mfbc_server_free of each of them. */
int mfbc_free_graph(mfbc_graph *g);

/*
 * mfbc_forward -- MFBF (Algorithm 1) for nb sources: tau and sigma.
 *   d_sources[nb]  device, vertex ids in [0,n); repeats allowed.
 *   d_dist[nb][n]  device out: tau(s,v), MFBC_INF_DIST if unreachable,
 *                  0 at the source.
 *   d_sigma[nb][n] device out: sigma(s,v) in binary64 (1 at the source,
 *                  0 if unreachable).
 *   h_products     host out (nullable): number of frontier products.
 * Errors: EINVAL (nb < 1, bad source), EOVERFLOW (a path count became
 * infinite), ENOMEM, EDEVICE.
 */
int mfbc_forward(mfbc_graph *g, const int32_t *d_sources, int32_t nb,
                 int32_t *d_dist, double *d_sigma, int32_t *h_products,
                 void *hip_stream);

/*
 * mfbc_backward -- MFBr (Algorithm 2) from a forward result: dependencies.
 *   d_sources[nb], d_dist[nb][n], d_sigma[nb][n]: as produced by
 *                  mfbc_forward for the same sources (device).
 *   d_delta[nb][n] device out: delta(s,v) = zeta(s,v) * sigma(s,v); 0 at the
 *                  source itself, at leaves and at unreachable vertices.
 *   h_products     host out (nullable): backward products, counting product
 *                  included.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int mfbc_backward(mfbc_graph *g, const int32_t *d_sources, int32_t nb,
                  const int32_t *d_dist, const double *d_sigma, double *d_delta,
                  int32_t *h_products, void *hip_stream);

/*
 * mfbc_bc -- MFBC (Algorithm 3): lambda over a list of sources.
 *   d_sources[n_sources] device; each occurrence counts once (a repeated
 *                  source contributes twice).  The full vertex set gives
 *                  exact betweenness; a subset gives the unscaled partial
 *                  sum sum_{s in S} delta(s,.).
 *   batch          sources per batch (n_b of Section 4); the last batch may
 *                  be smaller.  The result does not depend on it beyond
 *                  rounding.
 *   d_bc[n]        device out, overwritten.
 *   The batches are independent (Algorithm 3 sums their contributions), so
 *   up to four of them run at once on separate streams ("lanes", see
 *   mfbc_set_lanes), each lane with its own workspace; lane 0 uses
 *   hip_stream, the others library-owned streams ordered after the work
 *   already on hip_stream.  Lambda is summed in a fixed lane and batch order,
 *   so repeated calls with the same lane count are bitwise identical.
 * Errors: EINVAL (n_sources < 0, batch < 1, bad source), EOVERFLOW,
 * ENOMEM, EDEVICE.
 */
int mfbc_bc(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources,
            int32_t batch, double *d_bc, void *hip_stream);

/*
 * mfbc_set_lanes -- how many batches of one mfbc_bc call run at once (a
 * tuning knob; results differ only in floating-point summation order).
 *   lanes  1..4, or 0 (the default): four where a product of one batch is
 *          too small to fill the device (arcs * column groups <= 2^24), else one.
 * Each lane holds its own workspace (see the workspace note above).
 * Errors: EINVAL (lanes outside [0, 4]).
 */
int mfbc_set_lanes(mfbc_graph *g, int32_t lanes);

/*
 * mfbc_bc_requests -- Algorithm 3 for several source lists at once, one
 * lambda per list: d_out[r][v] = sum over the sources s of list r of
 * delta(s, v) (Section 4.3, the sum of Brandes' dependencies; a list's own
 * sources are excluded exactly as in mfbc_bc).  The lists share batches:
 * each list's sources take whole groups of 64 columns (its last group
 * padded), groups of all lists in order fill batches of `batch` columns,
 * and the lambda parts of each group go to its list's sum in ascending
 * group order -- several small lists cost one batch's products instead of
 * one batch each.
 *   d_sources   device int32[h_first[n_requests]]: the lists concatenated
 *               (caller vertex ids, repeats allowed);
 *   h_first     host int64[n_requests + 1]: list r is
 *               d_sources[h_first[r] .. h_first[r+1]), h_first[0] = 0,
 *               non-decreasing (empty lists give zero sums);
 *   batch       columns per batch: a multiple of 64 in [64, 4096];
 *   h_out       host array of n_requests device pointers, each to n
 *               doubles, overwritten (distinct lists need distinct outputs).
 * Synchronous on hip_stream.  Sums agree with mfbc_bc on the same list
 * within rounding (a different order of the additions).
 * Errors: EINVAL (bad lists, batch, NULL pointers, a source outside
 * [0, n)), EOVERFLOW, ENOMEM, EDEVICE.
 */
int mfbc_bc_requests(mfbc_graph *g, const int32_t *d_sources, const int64_t *h_first,
                     int32_t n_requests, int32_t batch, double *const *h_out, void *hip_stream);

/*
 * mfbc_bc_noalloc -- mfbc_bc for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results and errors as mfbc_bc, but the call
 * allocates nothing.  The batch state lives in a static scratch area of
 * 64 MiB per device, part of the library's code object (every GPU the library
 * runs on holds it until the process ends); the graph's own workspace is not
 * used or changed.  Sources are checked on the device.
 *   Limit: the state of one batch of min(batch, n_sources) sources must fit
 *   the scratch -- about 39 B per (source column, vertex), columns counted in
 *   whole groups of 64 (an even number of groups when there are two or more),
 *   plus 8 B per (group, arc) and the graph's hub partials; a larger request
 *   fails with MFBC_ENOMEM before any device work (n = 1024 with batches of
 *   256 fits; n = 65536 with batches of 512 does not).
 *   Every call on a device uses that device's one scratch area and leaves its
 *   contents behind: calls that overlap on one device (other threads, other
 *   streams) race and must be serialised by the caller.
 * Errors: as mfbc_bc (ENOMEM when the batch state exceeds the scratch).
 */
int mfbc_bc_noalloc(mfbc_graph *g, const int32_t *d_sources, int64_t n_sources,
                    int32_t batch, double *d_bc, void *hip_stream);

/*
 * mfbc_fixpoint -- the paper's monoid product (Section 3: C = A (+).f B with a
 * commutative monoid (+) and an action f of an arc on an entry) iterated over
 * maximal frontiers as in Algorithm 1, for other graph problems.  The
 * algebra is chosen by `op` (value type, (+), f):
 *   MFBC_OP_SSSP    int32, min, f(a, w) = a + w      -> shortest-path distances;
 *   MFBC_OP_BFS     int32, min, f(a, w) = a + 1      -> hop levels (weights ignored);
 *   MFBC_OP_WIDEST  int32, max, f(a, w) = min(a, w)  -> widest-path (bottleneck)
 *                   capacities; unweighted graphs have every width 1;
 *   MFBC_OP_RESIST  float (binary32), min, f(a, w) = a + 1/w -> the least sum of
 *                   reciprocal arc weights over paths, every division and
 *                   addition rounded to nearest (the value is the same for
 *                   any evaluation order: (+) is exact and f is monotone).
 * T(s,s) = 0 (MFBC_INF_DIST for WIDEST: the source's own width is
 * unbounded); product j relaxes the arcs of the entries that product j-1
 * improved (the sources for j = 1), an entry joining the next frontier when
 * the product improves it strictly in the order of (+); the loop ends after
 * the first product that improves nothing.  The product is the same
 * generic pull product MFBF's forward product runs.
 *   d_sources[nb]  device, vertex ids in [0,n) (repeats allowed), nb >= 1.
 *   d_out[nb][n]   device out, row-major, int32 (SSSP, BFS, WIDEST) or float
 *                  (RESIST); where v is unreachable from the source:
 *                  MFBC_INF_DIST (SSSP, BFS), 0 (WIDEST), +infinity (RESIST).
 *   h_products     host out (nullable): products run, the last one included.
 * Errors: EINVAL (op unknown, nb < 1, NULL output, bad source), ENOMEM,
 * EDEVICE.
 */
#define MFBC_OP_SSSP 0
#define MFBC_OP_BFS 1
#define MFBC_OP_WIDEST 2
#define MFBC_OP_RESIST 3
int mfbc_fixpoint(mfbc_graph *g, int32_t op, const int32_t *d_sources, int32_t nb,
                  void *d_out, int32_t *h_products, void *hip_stream);

/*
 * mfbc_forward_trace -- mfbc_forward that also records, after every forward
 * product j (Algorithm 1's loop; the frontier is the set of entries of the
 * product not heavier than what T held, Lemma 1 of Section 4.1.3), which
 * (source, vertex) pairs are in the new frontier F_j, and the work of each
 * product.  The first frontier F_0 (the sources themselves) precedes
 * product 1; the last product produces an empty frontier.
 *   d_fbits        device out (nullable): uint64 bitmaps [max_products][nb][W]
 *                  with W = (n + 63) / 64 words per row: bit v % 64 of word
 *                  v / 64 of row (j-1, s) is set iff caller vertex v is in F_j
 *                  of the s-th listed source.  Rows of products past the
 *                  last one (or all rows, if max_products exceeds it) are 0;
 *                  products past max_products are not recorded.
 *   max_products   rows of d_fbits and entries of h_nnz / h_relax (>= 0).
 *   h_nnz          host out (nullable): h_nnz[j-1] = |F_j| over all sources.
 *   h_relax        host out (nullable): h_relax[j-1] = relaxations of product
 *                  j = sum over the entries (s, u) of F_{j-1} of the number of
 *                  arcs leaving u (the flops of Section 5's cost model).
 *   other arguments and errors as mfbc_forward (EINVAL for max_products < 0).
 * Entries of h_nnz / h_relax past the last product are left untouched.
 */
int mfbc_forward_trace(mfbc_graph *g, const int32_t *d_sources, int32_t nb,
                       int32_t *d_dist, double *d_sigma, uint64_t *d_fbits,
                       int32_t max_products, int64_t *h_nnz, int64_t *h_relax,
                       int32_t *h_products, void *hip_stream);

/*
 * mfbc_backward_trace -- mfbc_backward that also records, for every
 * reachable (s,v), the index k of the backward frontier B_k it entered
 * (k = 0: leaves found by the counting product); -1 for unreachable.
 *   d_step[nb][n]  device out (int32).
 */
int mfbc_backward_trace(mfbc_graph *g, const int32_t *d_sources, int32_t nb,
                        const int32_t *d_dist, const double *d_sigma,
                        double *d_delta, int32_t *d_step,
                        int32_t *h_products, void *hip_stream);

/*
 * Work counters of the last forward/backward/bc/fixpoint call on a graph
 * (sums over its products; a fixpoint fills the forward fields).  "Entries" are frontier entries produced; "outputs" are
 * product entries that received a candidate; "active vertices/arcs" are the
 * vertices of the frontier a product read and the arcs of their rows.  The
 * *_ms fields are kernel times measured with HIP events recorded on the
 * call's stream around each launch; they are filled only while timing is
 * enabled (mfbc_enable_timing).  The *_alg_bytes fields are the bytes the
 * method must move (each frontier tuple, adjacency row and touched output
 * once per product; see the documentation of the measurement model).
 */
typedef struct mfbc_stats {
    int64_t fwd_products;   /* forward products over all batches          */
    int64_t bwd_products;   /* backward products (counting ones included)  */
    int64_t fwd_entries;    /* frontier entries produced, forward          */
    int64_t bwd_entries;    /* frontier entries produced, backward         */
    int64_t batches;
    int64_t fwd_outputs;
    int64_t bwd_outputs;
    int64_t fwd_active_vertices;
    int64_t fwd_active_arcs;
    int64_t bwd_active_vertices;
    int64_t bwd_active_arcs;
    int64_t fwd_pull_launches;
    int64_t bwd_pull_launches;
    int64_t count_launches;
    double fwd_pull_ms;     /* forward product kernel                      */
    double fwd_merge_ms;    /* merge of split rows, forward                */
    double count_ms;        /* counting product (both kernels)             */
    double bwd_pull_ms;     /* backward product kernel                     */
    double bwd_merge_ms;
    double other_ms;        /* initialisation and lambda reduction         */
    double fwd_alg_bytes;
    double bwd_alg_bytes;
    double count_alg_bytes;
} mfbc_stats;

/*
 * mfbc_set_plan -- choose the work decomposition of a graph's products (a
 * tuning knob; results do not depend on it).  Light rows are grouped into
 * runs of at most run_verts (1..64) rows and about run_arcs arcs; rows with
 * more than `heavy` arcs are cut into slices of `slice` arcs, merged in slice
 * order.  Any argument <= 0 restores the size-based default for that knob;
 * run_arcs, heavy and slice above 2^24 are rejected (EINVAL), and so is any
 * change while a server (mfbc_server_create) is attached to the graph.
 */
int mfbc_set_plan(mfbc_graph *g, int32_t run_arcs, int32_t run_verts, int32_t heavy,
                  int32_t slice);

/* Per-launch kernel timing of a graph: 0 off; 1 every product kernel and
 * merge (three events per product); 2 only the forward and fixpoint product
 * kernels (two events each: every event costs the stream a few
 * microseconds, which the steps of small graphs feel).  EINVAL otherwise. */
int mfbc_enable_timing(mfbc_graph *g, int enable);

int mfbc_get_stats(const mfbc_graph *g, mfbc_stats *out);

/* Graph facts: vertices, arcs, maximum weight. */
int mfbc_graph_info(const mfbc_graph *g, int32_t *n, int64_t *n_arcs,
                    int32_t *max_weight);

/*
 * mfbc_bc_many -- batched form: MFBC over many independent graphs in one
 * persistent launch.  Each workgroup takes (graph, job_width-source) jobs
 * from a device queue and runs Algorithms 1-3 for its job with no host
 * round trip per product; jobs are issued largest first.  Per graph the
 * result equals mfbc_bc(graphs[i], d_sources[i], h_n_sources[i], job_width,
 * d_bc[i]) up to rounding (the per-job parts are summed in job order, so
 * repeated calls with one configuration are bitwise identical).
 *   graphs[n_graphs]      host array of loaded graphs (same device).
 *   d_sources[n_graphs]   host array of device pointers to each graph's
 *                         source list; h_n_sources[n_graphs] their lengths.
 *   d_bc[n_graphs]        host array of device pointers, each [n_i], out.
 *   config (nullable)     launch shape: block_threads in {256, 512}
 *                         (0 = 512), blocks = persistent workgroups
 *                         (0 = enough for eight waves per SIMD on every
 *                         compute unit: 2048 / block_threads per CU); the
 *                         block count is capped so that the per-workgroup
 *                         state fits half of the device memory that is free
 *                         or already held by this call's workspace (the same
 *                         cap on every call);
 *                         job_width 64 or 128 sources per job (0 = 64):
 *                         128 runs the paired products (one gather per arc
 *                         for both column groups) at twice the state per
 *                         workgroup.
 *   h_stats (nullable)    out: products over all jobs.
 * The library keeps a grow-only workspace per device for this call, shared
 * by every call on that device: calls on one device must not overlap (one
 * host thread at a time), and the graphs of a call follow the one-thread rule
 * above for its duration.
 * Errors: EINVAL, ENOMEM, EOVERFLOW, EDEVICE.
 */
typedef struct mfbc_many_config {
    int32_t block_threads;
    int32_t blocks;
    int32_t job_width;
} mfbc_many_config;

int mfbc_bc_many(int32_t n_graphs, mfbc_graph *const *graphs,
                 const int32_t *const *d_sources, const int64_t *h_n_sources,
                 double *const *d_bc, const mfbc_many_config *config,
                 mfbc_stats *h_stats, void *hip_stream);

/*
 * Served form: continuous batching of source columns over a resident graph.
 *
 * A server owns `width` source columns (a positive multiple of 64) of one
 * graph; each column holds one source and moves through the phases forward
 * loop, counting product, backward loop, done.  A step runs the counting
 * product of the columns whose forward loop has ended, then R rounds of one
 * forward and one backward product (mfbc_server_set_rounds), advancing every
 * active column by up to R products of its phase; a column depends only on its own
 * column of the frontier (the products act column by column, Section 3), so
 * new sources start between steps while other columns are mid-loop.  The
 * unit of admission is a pair of 64-column groups (the last pair of a width
 * that is an odd multiple of 64 holds one group): a pair takes new sources
 * (from any number of requests) only while all of its columns are free or
 * until the step after its first admission is launched, and it leaves the
 * forward loop when all of its lanes have, so each pair follows the plain
 * path's per-batch schedule.  Finished columns are harvested into the
 * caller's buffers and become free.  All calls on one server must come from one
 * thread, in the order admit / step_launch / step_finish / harvest; the
 * stream argument must be the same for a step's launch and finish.
 */
typedef struct mfbc_server mfbc_server;

/* HBM bytes a server of `width` columns on graph g allocates. */
int mfbc_server_footprint(const mfbc_graph *g, int32_t width, int64_t *bytes);

/* Create a server (allocates its state; the graph must outlive it). */
int mfbc_server_create(mfbc_graph *g, int32_t width, mfbc_server **out);
int mfbc_server_free(mfbc_server *s);

/* Number of columns that can be admitted now (free columns of groups that
 * admit) / columns in a forward, counting or backward phase (>= 0), or a
 * negative status. */
int mfbc_server_free_columns(const mfbc_server *s);
int mfbc_server_active_columns(const mfbc_server *s);

/* Place `count` sources (host, in [0,n)) into admissible columns (groups
 * already opened since the last launch first); h_columns[i] receives the
 * column of source i.  EINVAL if fewer columns can be admitted. */
int mfbc_server_admit(mfbc_server *s, const int32_t *h_sources, int32_t count,
                      int32_t *h_columns, void *hip_stream);

/* Rounds of products per step: 1..8, or 0 (the default, 8).  More rounds:
 * fewer round trips to the host per product; fewer: new sources admitted
 * sooner.  EINVAL while a step is in flight or outside [0, 8]. */
int mfbc_server_set_rounds(mfbc_server *s, int32_t rounds);

/* Enqueue one step on the stream (does not wait). */
int mfbc_server_step_launch(mfbc_server *s, void *hip_stream);

/* 1 if no step is in flight or the launched one has completed, 0 if it is
 * still running, or a negative status (does not wait). */
int mfbc_server_step_query(mfbc_server *s);

/* Wait for the step and update the column phases; h_done[width] receives
 * the columns that finished in this step, *h_ndone their number.
 * EOVERFLOW if a shortest-path count of some column exceeded binary64: the
 * columns in flight then hold invalid results (free the server). */
int mfbc_server_step_finish(mfbc_server *s, int32_t *h_done, int32_t *h_ndone,
                            void *hip_stream);

/* Harvest finished columns into lambda-style sums:
 * d_dest[i][v] += delta(source of h_columns[i], v) for every v (device
 * buffers of n doubles; several columns may share one destination, which is
 * then updated column group by column group, ascending, and in list order
 * within a group).  The columns become free. */
int mfbc_server_harvest_bc(mfbc_server *s, const int32_t *h_columns, int32_t count,
                           double *const *d_dest, void *hip_stream);

/* Harvest finished columns as dependencies at target vertices:
 * d_out[i][t] = delta(source of h_columns[i], d_targets[t]) (d_targets:
 * device int32[ntargets]; d_out[i]: device double[ntargets]).  The columns
 * become free. */
int mfbc_server_harvest_dep(mfbc_server *s, const int32_t *h_columns, int32_t count,
                            const int32_t *d_targets, int32_t ntargets,
                            double *const *d_out, void *hip_stream);

/* Human-readable description of the last failure on this thread. */
const char *mfbc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFBC_H */
