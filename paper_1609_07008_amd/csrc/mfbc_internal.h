// Internal declarations of libmfbc (not part of the C ABI).
//
// Layout of the per-batch state in HBM ("column-group tiles"): the n_b
// source columns of a batch are cut into groups of 64, one per wavefront
// lane, and every per-(source, vertex) array is stored [cg][v][64]:
// element (cg, v, lane) at ((cg * n) + v) * 64 + lane.  A wave that owns
// (v, cg) touches 64 contiguous entries (256 B of int32, 512 B of double),
// and a launch that walks the column groups one after another keeps the
// working set of one group (n * 64 entries) hot in the 256 MB
// infinity cache.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mfbc.h"

namespace mfbc {

constexpr int kWave = 64;                // lanes per wavefront on CDNA
constexpr int kWavesPerBlock = 4;        // 256-thread workgroups
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int32_t kInf = MFBC_INF_DIST;
constexpr int kCounterSlots = 32;        // spread of the frontier-size counters
constexpr int kCounterRing = 16;         // products whose counters are live at once
constexpr int kWindow = 8;               // products enqueued per read-back of their counters
                                         // (at most kCounterRing - 1)
constexpr int kWide = 2;                 // column groups per wave in the forward product
constexpr int kMaxLanes = 4;             // batches of one mfbc_bc call run concurrently

// A unit of pull work for one wave (and one column group):
//  * hub < 0: the whole adjacency rows of vertices [v0, v1), arcs [e0, e1);
//  * hub >= 0: the slice [e0, e1) of vertex v0's row, written as partial
//    number `part`; a merge kernel combines the parts of the hub.
struct Task {
    int32_t v0, v1;
    int32_t hub, part;
    int64_t e0, e1;
};

struct Hub {
    int32_t v;       // vertex id
    int32_t first;   // first partial slot
    int32_t nparts;  // number of slices
    int32_t pad;
};

// Tunables of the work decomposition (chosen by the autotuner; defaults
// are used when none is set).
struct TaskParams {
    int run_arcs = 512;   // arcs per light run
    int run_verts = 64;   // vertices per light run (<= 64)
    int heavy = 1024;     // degree above which a row is split
    int slice = 512;      // arcs per slice of a split row
};

// Work decomposition of one CSR orientation.
struct Plan {
    Task *tasks = nullptr;   // device
    Hub *hubs = nullptr;     // device
    int32_t ntasks = 0, nhubs = 0, nslots = 0;
};

// Device CSR of one orientation (out-arcs or in-arcs).
struct Csr {
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    int32_t *w = nullptr;    // nullptr: unweighted (all 1)
    uint32_t *pk = nullptr;  // col | w << cb when both fit 32 bits (weighted only)
    int cb = 32;             // bits of a column index in pk
};

struct Workspace {
    int ncg = 0;                       // capacity in column groups
    int32_t *tdist = nullptr;          // T.w      [cg][n][64]
    double *tsig = nullptr;            // T.m      [cg][n][64]
    int32_t *fdist[2] = {nullptr, nullptr};  // frontier weights (double-buffered)
    double *fsig[2] = {nullptr, nullptr};    // frontier multiplicities
    uint64_t *fbits[2] = {nullptr, nullptr}; // frontier lane masks [cg][n]
    uint32_t *abits[2] = {nullptr, nullptr}; // activity bitmaps [cg][n/32] (backward: plane 0)
    int32_t *pd = nullptr;             // partial weights / counters [cg][slots][64]
    double *pm = nullptr;              // partial multiplicities / sums
    unsigned long long *counters = nullptr;  // [ring][4][slots]
    int32_t *flags = nullptr;          // [0]: path count overflow, [1]: source out of range
    double *lam = nullptr;             // per-column-group lambda parts [cg][n]
    int32_t *src = nullptr;            // column -> source vertex, -1 = padding
    uint64_t *dag = nullptr;           // shortest-path DAG: lane mask per out-arc [cg][arcs]
    uint32_t *tau2 = nullptr;          // tau per pair of groups, 16 bits a group [cg/2][n][64]
                                       // (read by the paired counting product)
    unsigned long long *trace_relax = nullptr;  // trace: relaxations per product
    int trace_len = 0;
    bool external = false;             // carved from caller-provided memory: never freed here
};

}  // namespace mfbc

struct mfbc_graph {
    int device = 0;
    int32_t n = 0;
    int64_t arcs = 0;
    int32_t maxw = 1;
    bool weighted = false;
    bool directed = false;
    mfbc::Csr out;          // out-arcs (backward products, counting product)
    mfbc::Csr in;           // in-arcs (forward products); aliases `out` if undirected
    mfbc::Plan plan_out, plan_in;
    int mb = 1;             // inline multiplicity bits of a packed frontier tuple
    mfbc::TaskParams params;
    mfbc::Workspace ws;
    mfbc_stats stats{};
    std::vector<int64_t> h_rp_out, h_rp_in;   // host copies for re-planning
    // Vertex order of the device copy: caller id v is stored as vertex perm[v]
    // (null / empty when the caller's order is kept).  Every entry point maps
    // sources through it and gathers per-vertex outputs back.
    int32_t *perm = nullptr;
    std::vector<int32_t> h_perm;
    int timing = 0;                    // kernel events: 0 off, 1 every product, 2 forward (and
                                       // fixpoint) product kernels only
    bool trace_step = false;           // backward products record frontier indices (traced call)
    hipEvent_t ev[3 * mfbc::kWindow] = {};   // per product of a window: before the product kernel,
                                       // between it and its merge, after the merge
    hipEvent_t ev_pull[3 * mfbc::kWindow] = {};  // timing 2: the first two of each, no merge event
    unsigned long long *h_ctr = nullptr;  // pinned host copy of the counter ring
    int servers = 0;                   // live mfbc_server objects on this graph
    // Lanes: mfbc_bc runs its batches on up to kMaxLanes streams at once, each
    // with its own workspace.  Lane 0 is the graph itself on the caller's
    // stream; lane i > 0 is a view (shadow) sharing the device graph and plans,
    // with its own workspace, counters, events and stream.
    int lanes = 0;                     // requested lanes (0: chosen by size)
    mfbc_graph *shadow[mfbc::kMaxLanes] = {};
    hipStream_t lane_stream[mfbc::kMaxLanes] = {};
    hipEvent_t lane_start = nullptr;   // recorded on the caller's stream, awaited by lanes
    bool is_shadow = false;
};

namespace mfbc {

// ---- launchers (kernels.hip) ----
void launch_fwd_init(mfbc_graph *g, int ncg, int nb, hipStream_t s);
// `ev` (nullable): three events recorded before the product kernel, between
// it and the merge kernel, and after the merge.  Product j (k) skips itself
// on the device when product j-1 (k-1) produced no frontier entry.
void launch_fwd_product(mfbc_graph *g, int ncg, int j, hipStream_t s, hipEvent_t *ev);
hipError_t launch_bwd_count(mfbc_graph *g, int ncg, hipStream_t s, hipEvent_t *ev);
void launch_bwd_product(mfbc_graph *g, int ncg, int k, hipStream_t s, hipEvent_t *ev);
// Trace: membership of forward frontier F_j (j = 0: the sources) as
// per-column vertex bitmaps in caller order (d_rows: nb rows of (n+63)/64
// words; nullable), and the out-degrees of its members added to
// ws.trace_relax[j] (the relaxations of product j+1).
void launch_trace_fwd(mfbc_graph *g, int ncg, int nb, int j, uint64_t *d_rows, hipStream_t s);
// Group slots of one batch of mfbc_bc_requests: the sources of each slot
// and the request sum its lambda parts go to.
constexpr int kMaxBatchGroups = 64;      // batches of up to 4096 columns
struct GroupSpans {
    int64_t first[kMaxBatchGroups];
    int32_t count[kMaxBatchGroups];
};
struct GroupOuts {
    double *out[kMaxBatchGroups];
};
void launch_set_sources_spans(mfbc_graph *g, int ncg, const int32_t *d_sources,
                              const GroupSpans &sp, hipStream_t s);
void launch_lambda_add_groups(mfbc_graph *g, int ncg, const GroupOuts &o, hipStream_t s);
void launch_zero_f64(double *p, size_t count, hipStream_t s);
void launch_lambda_zero(mfbc_graph *g, int ncg, hipStream_t s);
void launch_lambda_reduce(mfbc_graph *g, int ncg, double *d_bc, hipStream_t s);
// bc[v] = the lambda parts of every lane's workspace, summed lane by lane.
void launch_lambda_reduce_lanes(mfbc_graph *const *lanes, int nlanes, int ncg, double *d_bc,
                                hipStream_t s);
void launch_export_forward(mfbc_graph *g, int ncg, int nb, int32_t *d_dist, double *d_sigma,
                           hipStream_t s);
void launch_import_forward(mfbc_graph *g, int ncg, int nb, const int32_t *d_dist,
                           const double *d_sigma, hipStream_t s);
void launch_export_backward(mfbc_graph *g, int ncg, int nb, double *d_delta, int32_t *d_step,
                            hipStream_t s);
void launch_set_sources(mfbc_graph *g, int ncg, int nb, const int32_t *d_sources, hipStream_t s);
// *d_bad := 1 if a source is outside [0, n), else 0 (no host copy of the list).
void launch_check_sources(const int32_t *d_sources, int64_t count, int n, int32_t *d_bad,
                          hipStream_t s);
void launch_export_tiles_i32(mfbc_graph *g, int ncg, int nb, const int32_t *tiles, int32_t *d_rows,
                             hipStream_t s);

// ---- monoid fixpoints (monoid.hip) ----
bool mono_op_known(int op);
void launch_mono_init(mfbc_graph *g, int op, int ncg, int nb, hipStream_t s);
void launch_mono_product(mfbc_graph *g, int op, int ncg, int j, hipStream_t s, hipEvent_t *ev);

// ---- batched form (batched.hip) ----
struct ManyWorkspace;
size_t many_slot_bytes(int n_max, int slots_max, int64_t arcs_max, int w);
int launch_bc_many(std::vector<mfbc_graph *> &graphs, const std::vector<const int32_t *> &d_src,
                   const std::vector<int64_t> &n_src, const std::vector<double *> &d_bc,
                   int block_threads, int blocks, int w, hipStream_t s, ManyWorkspace &ws,
                   unsigned long long *h_stats, int32_t *h_flags, std::string &err);
ManyWorkspace &many_workspace(int device);

// Record the message of a failure for mfbc_last_error(); returns `code`.
int set_error(int code, const std::string &msg);

// ---- host helpers (graph.cpp) ----
TaskParams default_params(int32_t n, int64_t arcs);
int build_plan(int32_t n, const int64_t *rp, const TaskParams &p, std::vector<Task> &tasks,
               std::vector<Hub> &hubs, int32_t &nslots);

}  // namespace mfbc

namespace mfbc {
size_t ws_scratch_bytes_impl(const ManyWorkspace &ws);
}
inline size_t ws_scratch_bytes(const mfbc::ManyWorkspace &ws) { return mfbc::ws_scratch_bytes_impl(ws); }
