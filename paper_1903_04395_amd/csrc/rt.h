// Internal runtime state of libsc shared by runtime.cpp (contexts, graphs,
// templates, options, tracing), exec.cpp (passes, batches, hipGraph replay,
// autotuning), counts.cpp (exact counts, residues, the estimator),
// ablation_run.cpp (the pruning-ablation baselines) and serve.cpp (the
// serving loop).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "sc_internal.h"

namespace sc {

// Device memory from the context's allocator hook, with the stream it was
// allocated for (handed back to the hook when it is freed).
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
};

struct Graph {
    int64_t n = 0, nnz = 0;
    DevMem rp, ci;
    DevMem perm;                 // [n] caller id of each internal vertex (relabelled graphs)
    int64_t n_rows = 0;          // rows of every count table (relabelled graphs drop the
                                 // isolated vertices, whose rows are identically 0)
    int64_t max_deg = 0;
    std::vector<int64_t> deg_host;
    // rows with more than `seg` neighbours, for the current segment size
    int seg = 0;
    DevMem split_rows, split_items, slot;
    int64_t n_split = 0, n_split_items = 0;
    double split_nnz = 0;
    // the same for segment sizes used before (kept until unload, so passes
    // and captured graphs that read them stay valid)
    struct SavedBins {
        DevMem split_rows, split_items, slot;
        int64_t n_split = 0, n_split_items = 0;
        double split_nnz = 0;
    };
    std::map<int, SavedBins> saved_bins;
    int busy = 0;                // passes of the serving loop in flight on this graph
};

struct Template {
    int t = 0;
    std::vector<int32_t> edges;  // 2*(t-1), caller ids
    int root = -1;               // requested root (-1: planner chooses)
    bool explicit_plan = false;
    std::vector<int> child_ptr, child_idx;
    double aut = 1.0;
};

struct TableKey {
    int k, h, a;
    bool operator<(const TableKey &o) const { return std::tie(k, h, a) < std::tie(o.k, o.h, o.a); }
};

// Tuned execution knobs for one (graph, template, k, batch).
struct Tuned {
    int interleave = 0;
    int lds_max = 0;
    int seg = 0;
    int wave_row_max = -1;
    double ms = 0;
};
using TuneKey = std::tuple<int, int, int, int>;   // graph id, template id, k, batch

// What one pass computes.
struct PassSpec {
    Graph *g = nullptr;
    const Plan *P = nullptr;
    int k = 0;
    uint64_t seed = 0, first = 0;
    uint64_t mod = 0;              // 0: exact uint64 counts; else counts mod this prime
};

// Index tables of one pass copied into memory the caller provides (the
// allocation-free entry point); keyed as the context's table caches are.
struct StagedTables {
    std::map<TableKey, const uint32_t *> split;
    std::map<TableKey, const uint16_t *> unrank, rank;
};

// Device buffers one in-flight pass uses besides the resident graph and the
// index tables.  `gen` changes whenever one of them is reallocated (captured
// graphs that baked the old addresses are then discarded).  `staged`, when
// set, supplies every index table the pass reads (nothing is uploaded).
struct PassBuffers {
    DevMem arena, colbuf, xbuf, npre, desc;
    uint64_t gen = 0;
    const StagedTables *staged = nullptr;
};

struct GraphExecKey {
    int graph_id, tmpl_id, k, batch, interleave, lds_max, wave_row_max, seg, chain;
    uint64_t mod, bufgen;
    bool operator<(const GraphExecKey &o) const {
        return std::tie(graph_id, tmpl_id, k, batch, interleave, lds_max, wave_row_max, seg, chain, mod, bufgen) <
               std::tie(o.graph_id, o.tmpl_id, o.k, o.batch, o.interleave, o.lds_max, o.wave_row_max, o.seg,
                        o.chain, o.mod, o.bufgen);
    }
};

struct ServeState;   // serve.cpp

}  // namespace sc

struct sc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    sc_alloc_fn alloc = nullptr;
    sc_free_fn free_fn = nullptr;
    void *user = nullptr;
    uint64_t budget = 0;
    std::string err;
    int k = 0;
    uint64_t seed = 0;
    std::map<int, std::unique_ptr<sc::Graph>> graphs;
    std::map<int, std::unique_ptr<sc::Template>> tmpls;
    int next_graph = 1, next_tmpl = 1;
    std::map<sc::TableKey, sc::DevMem> split_tabs, unrank_tabs, rank_tabs;
    sc::PassBuffers main;                 // buffers of the synchronous calls
    sc::DevMem wide_tab, wide_x;          // exact multi-limb chain passes: output table, sums
    uint64_t *host_out = nullptr;         // pinned staging for results and descriptors
    size_t host_out_words = 0;
    std::map<sc::GraphExecKey, hipGraphExec_t> graph_cache;
    // SC_OPT_GRAPH = 2: one captured graph per call shape (every pass of an
    // sc_run / sc_run_batch call), reading per-pass descriptors from call_desc
    // and writing per-pass sums to call_x; call_gen changes when those move
    std::map<std::pair<std::vector<sc::GraphExecKey>, uint64_t>, hipGraphExec_t> call_graphs;
    sc::DevMem call_desc, call_x;
    uint64_t call_gen = 0;
    std::map<sc::TuneKey, sc::Tuned> tuned;
    // options
    int64_t max_batch = SC_MAX_BATCH, use_graph = 0, segment = 0;
    int64_t interleave = 0, lds_max = 0, wave_row_max = -1, reorder = 1, chain = 1;
    // tracing
    bool prof = false;
    struct Rec {
        const char *name;          // family
        std::string kernel;        // instantiation
        int step, h, a, p, colorings;
        hipEvent_t a_ev, b_ev;
        double bytes, layout_bytes, updates;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    // the serving loop and the lock it shares with the caller's thread
    std::recursive_mutex mu;
    sc::ServeState *serve = nullptr;      // owned; created by sc_serve_start, freed by serve_shutdown
};

namespace sc {

int fail(sc_ctx *c, int code, const char *fmt, ...);

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::sc::fail(ctx, SC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Memory from the allocator hook for use on `st` (NULL: the context's stream).
int dev_alloc(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st = nullptr);
void dev_free(sc_ctx *c, DevMem &m);
// Grows m to at least `bytes` (contents not kept); waits for `st` before freeing.
int ensure(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st, uint64_t *gen = nullptr);
int upload(sc_ctx *c, DevMem &m, const void *host, size_t bytes);
int host_staging(sc_ctx *c, size_t words);

int default_segment(const sc_ctx *c);
// The segment size a plan runs with (its tuned one, else the context's).
int plan_segment(const sc_ctx *c, const Plan &P);
// Makes `seg` the graph's current binning: switches to saved bins without
// allocating when they exist (allocate = false: fails with SC_ESTATE
// otherwise), else builds and uploads them.
int rebin(sc_ctx *c, Graph &g, int seg, bool allocate = true);
kern::GraphBins bins_of(const Graph &g);
// Device copies of the host index tables, cached per context.
int get_split(sc_ctx *c, int k, int h, int a, const uint32_t **out);
int get_unrank(sc_ctx *c, int k1, int s, const uint16_t **out);
int get_rank(sc_ctx *c, int k1, const uint16_t **out);

// Execution options for (graph, template, k, batch): context defaults,
// overridden by tuned values.
ExecOpts exec_opts(const sc_ctx *c, int gid, int tid, int k, int batch);
int make_plan(sc_ctx *c, const Graph &g, const Template &T, const ExecOpts &o, int k, int batch,
              Plan &P);
// Largest batch <= want whose pass fits `budget` bytes (0: the context budget).
int pick_batch(sc_ctx *c, int gid, int tid, int k, int want, uint64_t budget, Plan &P);
uint64_t pass_bytes(const Graph &g, const Plan &P);
double colorful_probability(int k, int t);

// Bytes `b` holds once a pass of plan P on graph g has run in it: buffers only
// grow, so each one ends at the larger of what it held and what P needs.
uint64_t buffers_after(const Graph &g, const Plan &P, const PassBuffers &b);
// Allocations and uploads a pass needs (not capturable).
int prepare_pass(sc_ctx *c, const PassSpec &s, PassBuffers &b, hipStream_t st);
// The pass's kernels on `st`, reading seed and first colouring from b.desc
// (capturable).  `prof` brackets launches with events.
int enqueue_pass(sc_ctx *c, const PassSpec &s, PassBuffers &b, hipStream_t st, bool prof);
// Everything for one pass on `st`: descriptor upload from host_desc[0..1],
// the kernels (direct or from a captured hipGraph), and the copy of
// SC_MAX_BATCH + 1 result words into host_res.
int launch_pass(sc_ctx *c, int gid, int tid, const PassSpec &s, PassBuffers &b, hipStream_t st,
                uint64_t *host_desc, uint64_t *host_res, bool allow_graph);
void unpack_pass(const uint64_t *host_res, int B, uint64_t *counts, uint8_t *flags);
// Mean-count estimates of maps and copies (NaN if any colouring overflowed).
void estimates(const uint64_t *counts, const uint8_t *ovf, int n, int k, int t, double aut,
               double *maps, double *copies);
// Bytes of the pre-pass neighbour sums of split rows for plan P on graph g.
size_t npre_bytes(const Graph &g, const Plan &P);
// Sets up the allocation-free entry point's device scratch on `device` (the
// device must be current); called once per context creation.
int static_scratch_init(int device);

// One pass of a planned job: colourings first..first+P.batch-1 of job `job`.
struct PassJob {
    int job, gid, tid, k;
    uint64_t seed, first;
    int offset;                // first colouring of this pass within its job
    uint64_t mod = 0;          // 0: uint64 counts with overflow flags; else residues mod this prime
    Plan P;
};
// Runs the passes back to back on `st` and waits once; then done(pass, its
// SC_MAX_BATCH + 1 result words) for each.
int run_passes(sc_ctx *c, std::vector<PassJob> &passes, hipStream_t st,
               const std::function<void(const PassJob &, const uint64_t *)> &done);
// Whether plan P is one chain from a single vertex covering every step (a
// star rooted at its centre), which the exact multi-limb kernels run.
bool single_chain(const Plan &P);
// Exact multi-limb counts of the colourings of passes with a single-chain
// plan, step i's entries kept as limbs[i] 64-bit limbs (launch_dp_chain_wide):
// each count's L = limbs.back() limbs (L + 1 words per colouring, the last
// the carry beyond) and a per-colouring flag mask, set where a carry left a
// step's top limb; waits for `st`.
int run_wide_passes(sc_ctx *c, std::vector<PassJob> &passes, const std::vector<int> &limbs, hipStream_t st,
                    const std::function<void(const PassJob &, const uint64_t *, uint64_t)> &done);
// SC_EINVAL unless colourings first..first+n-1 all lie below SC_MAX_COLORING.
int check_coloring_range(sc_ctx *c, uint64_t first, int64_t n);
// Splits n colourings of one job into passes of the planned batch.
int plan_job(sc_ctx *c, int job, int gid, int tid, int k, uint64_t seed, uint64_t first, int n,
             std::vector<PassJob> &out);
// Checks a run's graph, template, k >= t and colouring count; selects the device.
int check_run_args(sc_ctx *c, int gid, int tid, int ncol);

void serve_shutdown(sc_ctx *c);
// Destroys the whole-call graphs (SC_OPT_GRAPH = 2); the device must be idle
// or the graphs' last launches finished.
void drop_call_graphs(sc_ctx *c);

}  // namespace sc
