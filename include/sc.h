/*
 * sc.h -- C ABI of libsc: colour-coding tree subgraph counting on AMD MI355X
 * (gfx950).
 *
 * The method is the dynamic program of Chen et al., "A GraphBLAS Approach for
 * Subgraph Counting" (HPDC'19):
 *  - Section 2.1: random colouring with k >= t colours; template partitioning
 *    into an active child (keeps the root) and a passive child (rooted at the
 *    other end of a cut root edge); bottom-up DP over count tables with one row
 *    per graph vertex and one column per colour set of the sub-template's size;
 *    colourful-count / (k!/k^k) estimates the number of embeddings.
 *  - Section 3, Eq. 1: colour sets are indexed by the combinatorial number system.
 *  - Section 4.1-4.2, Eq. 2: the neighbour sum is taken once per passive colour
 *    set and stored (N = A * M_p, an SpMM over the 0/1 adjacency).
 *  - Section 4.5 (Algorithm 4): the rest of a step is an element-wise
 *    multiply-add ("eMA") M_s[v,C] = sum_{C1 (+) C2 = C} M_a[v,C1] * N[v,C2].
 *
 * Counts are exact unsigned 64-bit residues.  Overflow is not an error: each
 * colouring carries a flag that is 1 iff some usable neighbour-sum entry, some
 * product, some table entry or the final count, evaluated exactly from the
 * stored 64-bit operands, reached 2^64.  A neighbour-sum entry N[v][C2] is
 * usable iff C2 leaves out the colour of v: every other entry only ever meets
 * zero active entries (the active child's root maps to v, so its colour set
 * holds col(v), and the split sets are disjoint).  The flag depends on the
 * plan (root and child order)
 * but not on summation order, batching or fusion; the residue depends on
 * nothing but (graph, template, k, seed, colouring index).  sc_run_exact
 * recovers the counts that pass 2^64 exactly (residue passes modulo primes and
 * the Chinese remainder theorem), and sc_estimate turns exact counts into an
 * (eps, delta) estimate.
 *
 * Colouring rule (the paper only says "randomly selected"): colouring r of
 * vertex v is floor(x * k / 2^64) where x is output number r*2^40 + v of
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) seeded with the context seed.
 * Vertex ids are below 2^31, so the rule gives distinct outputs for colouring
 * indices below SC_MAX_COLORING = 2^24; every call that runs colourings
 * rejects a range that reaches past it (SC_EINVAL), because colouring
 * r + 2^24 would repeat colouring r and the colourings would no longer be
 * independent draws.
 *
 * Conventions for every call:
 *  - return value: SC_OK (0) or a negative SC_E* code; nothing throws or aborts;
 *    sc_last_error() then holds a message (owned by the context, valid until the
 *    next call on the same context).
 *  - pointer arguments documented as "host" are read or written during the call
 *    only; the caller keeps ownership.  Device memory that the library allocates
 *    belongs to the context until the matching unload/destroy.
 *  - a context is used by one host thread at a time, except the serving calls
 *    (sc_serve_*), which are internally synchronised.
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SC_MAX_T 16          /* template vertices */
#define SC_MAX_K 16          /* colours */
#define SC_MAX_BATCH 64      /* colourings folded into one pass */
#define SC_MAX_COLORING (1ull << 24)   /* colouring indices run below this */

enum {
    SC_OK = 0,
    SC_EINVAL = -1,     /* malformed argument, graph or template */
    SC_ENOMEM = -2,     /* device allocation failed or plan exceeds the budget */
    SC_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed */
    SC_ENOTFOUND = -4,  /* unknown graph / template id or ticket */
    SC_EBUSY = -5,      /* result not ready yet (sc_poll) */
    SC_ESTATE = -6      /* call not valid in the current state */
};

typedef struct sc_ctx sc_ctx;

/* Device allocator hook, required: every device buffer the library holds
 * (resident graphs, index tables, count tables, colours, results) comes from
 * `alloc` and goes back through `free_fn`; the library never allocates device
 * memory any other way.  `alloc` returns device memory of at least `bytes`
 * bytes for use on `stream` (a hipStream_t), or NULL on failure (the call
 * that needed it then returns SC_ENOMEM); `free_fn` receives the pointer, its
 * size and the stream it was allocated for, once the library's work on it has
 * completed.  The hooks may be called from the serving loop's worker thread.
 * The Python binding passes PyTorch's caching allocator. */
typedef void *(*sc_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*sc_free_fn)(void *ptr, size_t bytes, void *stream, void *user);

/* Creates a context on HIP device `device` with the allocator hooks `alloc` /
 * `free_fn` (both required; `user` is passed to them).  `mem_budget_bytes`
 * caps the count tables of one run (0 = 90% of the device's free memory at
 * creation).  The context owns a non-blocking stream of its own, which every
 * call given a NULL stream uses.
 * Errors: SC_EINVAL (bad device, NULL alloc or free_fn), SC_EDEVICE. */
int sc_create(int device, sc_alloc_fn alloc, sc_free_fn free_fn, void *user,
              uint64_t mem_budget_bytes, sc_ctx **out);

/* Releases every device buffer owned by the context (after draining the
 * serving loop if it runs), then the context.  NULL is accepted. */
int sc_destroy(sc_ctx *ctx);

/* Message for the last failed call on `ctx` (empty string if none). */
const char *sc_last_error(const sc_ctx *ctx);

/* Library version string, static storage. */
const char *sc_version(void);

/* ------------------------------------------------------------------ inputs */

/* Loads a simple undirected graph as its symmetric 0/1 adjacency A_G in CSR
 * form (the paper stores A_G in CSC, Section 4.3; for a symmetric matrix the
 * two coincide).  Host arrays: row_ptr[n+1] (int64, row_ptr[0]=0,
 * non-decreasing, row_ptr[n]=nnz), col_idx[nnz] (int32 in [0,n), strictly
 * increasing within a row, no self-loops, and (i,j) present iff (j,i) is).
 * The arrays are validated, copied to the device and kept resident.
 * Errors: SC_EINVAL (any rule above broken; n < 1 or n >= 2^31), SC_ENOMEM,
 * SC_EDEVICE. */
int sc_load_graph_csr(sc_ctx *ctx, int64_t n, int64_t nnz, const int64_t *row_ptr,
                      const int32_t *col_idx, int32_t *graph_id);

int sc_unload_graph(sc_ctx *ctx, int32_t graph_id);

/* Loads a template tree T: t vertices 0..t-1 (1 <= t <= SC_MAX_T) and t-1
 * undirected edges given as host int32 pairs edges[2*i], edges[2*i+1].
 * `root` selects the root of the partitioning (Section 2.1, phase 2), or -1 to
 * let the planner choose the root and child order with the lowest modelled
 * cost.  Errors: SC_EINVAL (not a tree, ids out of range, bad root). */
int sc_load_template(sc_ctx *ctx, int32_t t, const int32_t *edges, int32_t root,
                     int32_t *tmpl_id);

/* Loads a template with an explicit plan: `child_ptr[t+1]`, `child_idx[t-1]`
 * list the children of every vertex in attach order (CSR form of a rooted,
 * ordered tree with root `root`).  Each attach of a child w to u is one DP step
 * (active child = the part of u's subtree built so far, passive child = the
 * subtree of w).  Errors: SC_EINVAL (not a rooted spanning tree). */
int sc_load_template_plan(sc_ctx *ctx, int32_t t, int32_t root, const int32_t *child_ptr,
                          const int32_t *child_idx, int32_t *tmpl_id);

/* Sets the number of colours k (t <= k <= SC_MAX_K, checked at run time) and
 * the colouring seed.  Errors: SC_EINVAL (k < 1 or k > SC_MAX_K). */
int sc_set_colors(sc_ctx *ctx, int32_t k, uint64_t seed);

/* ------------------------------------------------------------------ plans */

typedef struct {
    int32_t t, k, root, n_steps;
    int32_t child_ptr[SC_MAX_T + 1];     /* rooted ordered tree (CSR)        */
    int32_t child_idx[SC_MAX_T];
    int32_t step_h[SC_MAX_T];           /* steps in execution order:        */
    int32_t step_a[SC_MAX_T];           /*   sizes of T_s, T_a, T_p         */
    int32_t step_p[SC_MAX_T];
    int32_t step_mode[SC_MAX_T];        /* 0: p = 1, neighbours' colours counted;
                                           1: p >= 2, neighbours' rows summed
                                           (both fused with the multiply-add) */
    int32_t batch;                      /* colourings per pass              */
    int32_t interleave;                 /* colourings interleaved per table
                                           plane (power of two dividing batch) */
    uint64_t arena_bytes;               /* device tables of one pass        */
    double spmm_updates;                /* per colouring: sum nnz*C(k,p)    */
    double ema_updates;                 /* per colouring: sum n*C(k,h)*C(h,a),
                                           n*C(k,h) for a = 1 (a select)    */
    double lemma1_ops;                  /* per colouring: Lemma 1,
                                           sum nnz*C(k,p) + n*C(k,h)*C(h,p) */
    double exec_updates;                /* per colouring, executed in the
                                           rooted-colour layout: sum
                                           nnz*C(k-1,p-1) + n*C(k-1,h-1)*C(h-1,a-1) */
    double compulsory_bytes;            /* per colouring, HBM bytes (model) */
    double automorphisms;               /* |Aut(T)|                         */
} sc_plan_info_t;

/* Pure host call (no device needed): plans template (t, edges, root as in
 * sc_load_template) for a graph of n vertices and nnz nonzeros, k colours and
 * `batch` colourings per pass, and fills `out`.  Lemma 1 gives the per-step
 * operation counts: nnz*C(k,p) neighbour-sum updates and n*C(k,h)*C(h,a)
 * multiply-adds.  Errors: SC_EINVAL. */
int sc_plan_template(int32_t t, const int32_t *edges, int32_t root, int32_t k, int64_t n,
                     int64_t nnz, int32_t batch, sc_plan_info_t *out);

/* Plan of a loaded template for a loaded graph, with the batch the library
 * would use for `n_colorings` colourings under the memory budget. */
int sc_plan_info(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, int32_t n_colorings,
                 sc_plan_info_t *out);

/* Pure host helpers exposing the library's own colour-set indexing (Eq. 1) and
 * colouring rule, for tests. */
int64_t sc_colorset_rank(uint32_t mask);
int32_t sc_color_of(uint64_t seed, uint64_t coloring, uint64_t vertex, int32_t k);

/* ------------------------------------------------------------------ runs */

/* Counts colourful maps of the template into the graph for colourings
 * first_coloring .. first_coloring+n_colorings-1 (colourings are folded into
 * the table columns, up to the planned batch per pass).  Synchronous: on return
 * the host outputs are written.  `stream` is a hipStream_t (NULL = the
 * context's own stream; the legacy null stream is not used because it cannot
 * be captured into a hipGraph).  Buffers the run allocates are requested
 * for this stream.
 * Host outputs: counts[n_colorings] (residues mod 2^64), overflow[n_colorings]
 * (0/1), and optionally (may be NULL) est_maps / est_copies: the mean count
 * divided by k!/((k-t)! k^t), and that divided by |Aut(T)|; NaN if any
 * colouring overflowed.
 * Errors: SC_EINVAL (k < t, n_colorings < 0), SC_ENOTFOUND, SC_ENOMEM, SC_EDEVICE. */
int sc_run(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, uint64_t first_coloring,
           int32_t n_colorings, void *stream, uint64_t *counts, uint8_t *overflow,
           double *est_maps, double *est_copies);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation between set-up and tear-down): sc_run with
 * every buffer of the run -- colours, count tables, the split rows' neighbour
 * sums, index tables, descriptor and results -- placed in one device array of
 * SC_STATIC_SCRATCH_BYTES that the library holds per device (and per process)
 * from its first sc_create on that device until the process ends.  The call
 * allocates nothing (no hipMalloc, no allocator hook, no pinned host memory);
 * the graph and template must already be loaded.  Same arguments, outputs,
 * counts and flags as sc_run; colourings are folded into passes whose
 * buffers fit the array.  Calls on one device are serialised inside the
 * process (the array keeps the last call's contents; everything a run reads
 * is written by that run first).  Synchronous.
 * Errors: as sc_run; SC_ENOMEM when even one colouring's buffers exceed
 * SC_STATIC_SCRATCH_BYTES; SC_ESTATE when the graph has no heavy-row bins for
 * the run's segment size (SC_OPT_SEGMENT or a tuned segment size not yet
 * used by sc_run on this graph: building the bins would allocate). */
#define SC_STATIC_SCRATCH_BYTES 67108864ull   /* 64 MiB */
int sc_run_static(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, uint64_t first_coloring,
                  int32_t n_colorings, void *stream, uint64_t *counts, uint8_t *overflow,
                  double *est_maps, double *est_copies);

/* Exact wide counts.  The DP uses only additions and multiplications, so it
 * commutes with reduction modulo any m (Eq. 2 and the counting recursion of
 * Sec. 2.1 with every entry taken mod m).  sc_run gives each count mod 2^64 and
 * flags the colourings whose count reached 2^64; for those, sc_run_exact adds
 * passes modulo the primes 2^61-1, 2^62-57, 2^63-25 and recovers the count by
 * the Chinese remainder theorem.  The homomorphism count of the template into
 * the graph bounds every colouring's colourful count; the first one, two or
 * three primes run, as that bound (with a 2^-10 margin) lies below 2^124,
 * 2^185 or 2^247, and the result is certified exact when it does.
 * A template that is one chain of single-vertex attaches from a single vertex
 * (the star rooted at its centre; SC_OPT_CHAIN on) skips the residue passes
 * when its bound reaches 2^64: one pass keeps each step's table entries as
 * 1 to 4 little-endian 64-bit limbs, the fewest that hold that step's bound
 * (the largest homomorphism count of its sub-star at any vertex, with the
 * same margin; the last step at least what the total bound needs), and the
 * counts are exact without any modular step (a bound at or past 2^256, or
 * rows too wide for the LDS limit, take the residue passes).  The
 * homomorphism count is then always computed.
 * Synchronous.  Host outputs: counts[n_colorings][4] (the count as four uint64
 * limbs, least significant first), exact[n_colorings] (1: the count is exact;
 * 0: only its residue mod 2^64 p1 p2 p3 is), hom_bound (may be NULL: the
 * homomorphism count, computed when a colouring overflowed, when asked for
 * or for a single-chain template, else NaN), est_maps / est_copies (may be NULL; from the exact counts, NaN if
 * any is not exact).
 * Errors: as sc_run. */
int sc_run_exact(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, uint64_t first_coloring,
                 int32_t n_colorings, void *stream, uint64_t *counts, uint8_t *exact,
                 double *hom_bound, double *est_maps, double *est_copies);

/* Estimates to relative error eps with probability at least 1 - delta.  The
 * paper bounds the colourings an (eps, delta)-approximation takes by
 * O(e^k log(1/delta) / eps^2) (Lemma 3 and its proof); here the constants come
 * from the median of means: the count estimate X/P of one colouring (P the
 * colourful probability, Sec. 2.1 phase 1) is unbiased with relative variance
 * at most 1/P - 1, so a mean of g >= 4 (1/P - 1) / eps^2 colourings misses by
 * more than eps with probability at most 1/4 (Chebyshev), and the median of
 * m >= 8 ln(1/delta) such means (m odd) misses with probability at most delta
 * (Hoeffding).
 * sc_colorings_for: m (groups) and g (per_group) of that bound, pure host.
 *   Errors: SC_EINVAL (eps <= 0, delta outside (0, 1), k < t, k > SC_MAX_K).
 * sc_estimate: runs colourings first_coloring, first_coloring + 1, ... with
 *   exact counts (as sc_run_exact) and returns the median of the means of m
 *   groups of consecutive colourings.  mode SC_EST_BOUND runs m * g colourings
 *   of the bound (SC_EINVAL if that exceeds max_colorings > 0); mode
 *   SC_EST_SAMPLE uses the sample relative variance in place of 1/P - 1,
 *   re-evaluated after each round (the first round 4m colourings, each round at
 *   most doubling the total), and stops when enough colourings ran or at
 *   max_colorings (> 0) -- a heuristic: the variance is estimated, not bounded.
 *   Synchronous.  Errors: as sc_run_exact, SC_EINVAL for bad eps/delta/mode or
 *   0 < max_colorings < m. */
enum { SC_EST_BOUND = 0, SC_EST_SAMPLE = 1 };
typedef struct {
    double est_maps, est_copies;   /* median of group means; NaN if a count is not exact */
    double mean_maps;              /* mean over every colouring run */
    double rel_stderr;             /* sample standard error of mean_maps, relative */
    int64_t colorings;             /* colourings run */
    int64_t per_group;             /* colourings per group used by the median */
    int64_t needed;                /* colourings the rule asked for at the end */
    int32_t groups;
    int32_t exact;                 /* 1: every count exact */
} sc_estimate_t;
int sc_colorings_for(int32_t k, int32_t t, double eps, double delta, int32_t *groups, int64_t *per_group);
int sc_estimate(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, uint64_t first_coloring, double eps,
                double delta, int32_t mode, int64_t max_colorings, void *stream, sc_estimate_t *out);

/* Baselines for the pruning ablation (Sec. 3.1, Sec. 4.1, Sec. 7.1): the same
 * counts as sc_run, one colouring at a time, by plain kernels over tables in
 * the paper's layout (all binom(k, s) colour sets per row):
 *   SC_ABL_FASCIA  -- Algorithm 1: every split sums the passive column over
 *                     the row's neighbours again;
 *   SC_ABL_PFASCIA -- pruned: each passive column's neighbour sum once per row,
 *                     then the split multiply-add.
 * Allocates every table of the plan for the call (no reuse).  Synchronous.
 * Host outputs as sc_run (counts, overflow).  Errors: as sc_run, SC_EINVAL for
 * an unknown variant. */
enum { SC_ABL_FASCIA = 1, SC_ABL_PFASCIA = 2 };
int sc_run_ablation(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, int32_t variant, uint64_t first_coloring,
                    int32_t n_colorings, void *stream, uint64_t *counts, uint8_t *overflow);

/* Residues: residues[r] = (colourful count of colouring first_coloring + r) mod p,
 * for p = 2^w - c with 61 <= w <= 63 and odd c <= 2^16 (p need not be prime).
 * Synchronous.  Errors: SC_EINVAL (unsupported p, NULL output), else as sc_run. */
int sc_run_mod(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, uint64_t first_coloring,
               int32_t n_colorings, void *stream, uint64_t p, uint64_t *residues);

/* Homomorphisms of the template into the graph (maps of the template's
 * vertices to the graph's that send edges to edges, not necessarily
 * injective), in double precision (relative error below 2^-40), by the same
 * steps as the counting DP (Sec. 2.1 phase 3) on one value per vertex with the
 * colour condition dropped.  Not a quantity of the paper: it bounds every
 * colouring's colourful count, which certifies sc_run_exact.  Synchronous.
 * Errors: SC_EINVAL (NULL output), SC_ENOTFOUND, SC_ENOMEM, SC_EDEVICE. */
int sc_hom_count(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, void *stream, double *out);

/* Batched form: many jobs -- each a (graph, template, k, seed, colouring range)
 * -- planned together and run back to back on one stream with a single host
 * wait at the end (colourings folded into the table columns, up to the
 * planned batch per pass; with SC_OPT_GRAPH = 1 each pass replays a captured
 * hipGraph, with SC_OPT_GRAPH = 2 the whole call does).  Jobs may mix templates of different sizes and different k.
 * Host outputs per job: counts[n_colorings], overflow[n_colorings],
 * est_maps / est_copies (NaN if any colouring overflowed), status.
 * Returns SC_OK, or the first job's error (that job's status is set, the
 * others still run). */
typedef struct {
    int32_t graph_id, tmpl_id, k;
    uint64_t seed, first_coloring;
    int32_t n_colorings;
    uint64_t *counts;
    uint8_t *overflow;
    double est_maps, est_copies;   /* out */
    int32_t status;                /* out */
} sc_job_t;
int sc_run_batch(sc_ctx *ctx, sc_job_t *jobs, int32_t n_jobs, void *stream);

/* Autotuner: times real passes of (graph, template) at the batch `n_colorings`
 * plans to, over the interleave caps {1, 2, 4, ..., batch} (at most four of
 * them, the largest ones) times the row-kernel LDS limits {32, 64, 96, 128} KB;
 * then, around the fastest, the neighbours per split-row work item {256, 512,
 * 1024, 2048}; then the per-row LDS up to which a wavefront builds a row alone
 * {0, 8192, 16384} bytes; and keeps the fastest for that (graph, template, k,
 * batch).  The choice never changes a result. */
typedef struct {
    int32_t interleave, lds_max, batch, trials;
    double ms;                      /* time of one pass with the chosen knobs */
    int32_t seg, wave_row_max;      /* the chosen segment size and row threshold */
} sc_tune_t;
int sc_autotune(sc_ctx *ctx, int32_t graph_id, int32_t tmpl_id, int32_t n_colorings, sc_tune_t *out);
/* Tuning cache as text lines keyed by graph shape (n, nnz, max degree),
 * template edges, k and batch.  Load applies entries to loaded graphs and
 * templates that match; *n_applied (may be NULL) counts them. */
int sc_tune_save(sc_ctx *ctx, const char *path);
int sc_tune_load(sc_ctx *ctx, const char *path, int32_t *n_applied);

/* ------------------------------------------------------------------ serving */

/* Serving loop with continuous batching.  A worker thread owns `max_inflight`
 * HIP streams.  Submitted queries wait in FIFO order; whenever a stream is
 * free, the head query gets a pass of as many of its colourings as fit the
 * device memory still free under `mem_budget_bytes` (0 = the context budget),
 * so a query that arrives while others run starts as soon as a stream and
 * memory free up, and passes of different queries overlap on the device.
 * Results do not depend on how a query was split or what ran beside it.
 * sc_serve_start first releases the count tables the synchronous calls keep
 * (a later sc_run allocates them again), so that the budget is the loop's.
 * sc_submit / sc_poll / sc_serve_stats may be called from any thread;
 * sc_serve_stop waits for every submitted query (poll results first: stop
 * discards them).  While the loop runs, options other than SC_OPT_GRAPH
 * cannot change and graphs with passes in flight cannot be unloaded. */
typedef struct {
    uint64_t mem_budget_bytes;
    int32_t max_inflight;           /* streams, 1..4 (HIP's default hardware
                                       queues per process; more streams would
                                       only share them) */
    int32_t max_batch;              /* colourings per pass, 1..SC_MAX_BATCH */
} sc_serve_cfg_t;

typedef struct {
    int32_t graph_id, tmpl_id, k;
    uint64_t seed, first_coloring;
    int32_t n_colorings;            /* >= 1 */
} sc_query_t;

typedef struct {
    int32_t status;                 /* SC_OK or the query's error */
    int32_t n_colorings;
    uint64_t *counts;               /* caller buffers of n_colorings (or NULL) */
    uint8_t *overflow;
    double est_maps, est_copies;
    double submit_s, start_s, done_s;   /* steady-clock seconds */
} sc_result_t;

typedef struct {
    uint64_t passes, colorings;
    int32_t waiting, inflight;
    uint64_t mem_bytes, peak_mem_bytes;
} sc_serve_stats_t;

int sc_serve_start(sc_ctx *ctx, const sc_serve_cfg_t *cfg);
int sc_submit(sc_ctx *ctx, const sc_query_t *query, uint64_t *ticket);
/* SC_EBUSY until the query is done; then fills *out (copying counts and
 * overflow into the caller's buffers) and releases the ticket. */
int sc_poll(sc_ctx *ctx, uint64_t ticket, sc_result_t *out);
int sc_serve_stats(sc_ctx *ctx, sc_serve_stats_t *out);
int sc_serve_stop(sc_ctx *ctx);

/* Execution options (for measurement and ablation; none changes a result).
 * Errors: SC_EINVAL (unknown option or value out of range). */
enum {
    SC_OPT_MAX_BATCH = 1,     /* cap on colourings per pass (1..SC_MAX_BATCH)   */
    SC_OPT_GRAPH = 3,         /* 1: replay each pass from a captured hipGraph;
                                 2: capture every pass of an sc_run /
                                 sc_run_batch call (templates, sizes and k
                                 mixed) into one hipGraph, replayed with one
                                 launch whenever a call of the same shape
                                 (passes, plans, knobs) comes again; serving
                                 treats 2 as 1                                 */
    SC_OPT_SEGMENT = 5,       /* neighbours per work item of heavy rows, > 64
                                 (0 = default, 512)                            */
    SC_OPT_REORDER = 8,       /* graphs loaded afterwards are kept relabelled:
                                 1 (default) by descending degree, 2 in reverse
                                 Cuthill-McKee order, 0 not at all (colours
                                 always follow the caller's vertex ids)        */
    SC_OPT_INTERLEAVE = 9,    /* cap on colourings interleaved per table plane:
                                 1, 2, 4, ..., 64 (0 = default, no cap)        */
    SC_OPT_LDS_MAX = 10,      /* LDS bytes per row-kernel workgroup,
                                 16384..163840 (0 = default, 65536)            */
    SC_OPT_WAVE_ROW_MAX = 11, /* steps whose per-row LDS is at most this many
                                 bytes build one row per wavefront instead of
                                 one per workgroup: 0..40960 (0 = never,
                                 -1 = default, 8192)                          */
    SC_OPT_CHAIN = 12         /* 1 (default): a run of steps that each attach a
                                 single vertex to the previous step's output
                                 runs as one kernel, its intermediate tables
                                 kept in LDS (when its two widest rows fit the
                                 LDS limit); 0: one kernel and table per step */
};
int sc_set_option(sc_ctx *ctx, int32_t option, int64_t value);
int sc_get_option(sc_ctx *ctx, int32_t option, int64_t *value);

/* ------------------------------------------------------------------ tracing */

/* Per-kernel-family statistics gathered with HIP events recorded around every
 * launch on the run's stream while profiling is on (families: zero, color,
 * split, row_hist, row_gather, reduce).  Summed over those launches:
 *  - alg_bytes: the algorithmic (compulsory) bytes of the method in the
 *    paper's table layout (binom(k, s) colour sets per row, every vertex of
 *    the graph; Sec. 4.3): per DP step (h, a, p) with B colourings,
 *    4 nnz + 8 (n+1) (the adjacency once), + 8 n B binom(k, p) (the passive
 *    table read once; n B colour bytes for p = 1), + 8 n B binom(k, a) (the
 *    active table; n B colour bytes for a = 1), + 8 n B binom(k, h) (the output
 *    written once).  The neighbour sum N of a fused step is never stored, so
 *    its write and read are not counted.  A step's bytes are attributed to
 *    its row kernel; the split pre-pass (rows with more neighbours than the
 *    segment size) carries none.
 *  - layout_bytes: the same in this library's rooted-colour layout
 *    (binom(k-1, s-1) sets per table row, non-isolated rows only), plus the
 *    split pre-pass's partial sums written and read back.
 *  - updates: Lemma 1's counts, nnz binom(k, p) neighbour-sum updates plus
 *    n binom(k, h) binom(h, a) multiply-adds (n binom(k, h) for a = 1), times B. */
typedef struct {
    char name[32];
    int32_t launches;
    double total_ms;
    double alg_bytes;
    double updates;
    double layout_bytes;
} sc_kernel_stat_t;

/* One traced launch: the kernel instantiation as profilers name it (e.g.
 * "dp_row_kernel<16, 1, false, 0, true, false, 256>"), its family, the DP step
 * it belongs to (index in the plan and its sizes h, a, p; step -1 outside the
 * steps), the colourings of its pass, its duration between HIP events on the
 * run's stream, and its bytes and updates as in sc_kernel_stat_t. */
typedef struct {
    char kernel[96];
    char family[16];
    int32_t step, h, a, p, colorings;
    double ms;
    double alg_bytes;
    double layout_bytes;
    double updates;
} sc_launch_t;

/* The vector-ALU roof of the multiply-add (the arithmetic of Algorithm 4's
 * element-wise multiply-add, exact 64-bit with overflow detection): every
 * wavefront slot of the device runs independent chains of multiply-adds on
 * register operands, timed with HIP events on `stream` (NULL = the context's).
 * form 0: the 128-bit product; 1: three 32-bit multiplies (the form of
 * vector-ALU-bound steps); 2: a second operand below 2^32 (the form of steps
 * whose passive child is one vertex).  Writes multiply-adds per second to
 * *mul_adds_per_s.  Allocates one word per thread through the hook for the
 * call.  Errors: SC_EINVAL (form outside 0..2, NULL output), SC_ENOMEM,
 * SC_EDEVICE. */
int sc_valu_probe(sc_ctx *ctx, int32_t form, void *stream, double *mul_adds_per_s);

/* enable = 1 starts recording (and clears earlier records), 0 stops. */
int sc_profile(sc_ctx *ctx, int32_t enable);
/* Waits for the recorded launches, aggregates them by family into out[0..cap)
 * and sets *n_out to the number of families.  Records are kept until the next
 * sc_profile(ctx, 1). */
int sc_profile_read(sc_ctx *ctx, sc_kernel_stat_t *out, int32_t cap, int32_t *n_out);
/* Waits for the recorded launches and copies the first `cap` of them, in
 * launch order, into out; *n_out = the number recorded. */
int sc_profile_launches(sc_ctx *ctx, sc_launch_t *out, int32_t cap, int32_t *n_out);

#ifdef __cplusplus
}
#endif
#endif /* SC_H */
