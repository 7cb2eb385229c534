// libsc runtime: contexts, resident graphs and templates, the per-pass DP
// executor and the C ABI of include/sc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "sc_internal.h"

using namespace sc;

namespace {

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Graph {
    int64_t n = 0, nnz = 0;
    DevMem rp, ci;
    DevMem perm;                             // [n] original id of each internal vertex (relabelled graphs)
    int64_t n_rows = 0;                      // rows of every count table (relabelled graphs
                                             // drop the isolated vertices, whose rows are 0)
    std::vector<int64_t> deg_host;           // degrees, for re-binning
    // bins for the current segment size
    int seg = 0;
    DevMem light, wide, split_rows, slot, tasks;
    int64_t n_light = 0, n_wide = 0, n_split = 0, n_split_items = 0, n_tasks = 0, n_split_tasks = 0;
};

struct Template {
    int t = 0;
    std::vector<int32_t> edges;     // 2*(t-1)
    int root = -1;                  // requested root (-1: planner)
    bool explicit_plan = false;
    std::vector<int> child_ptr, child_idx;
    double aut = 1.0;
};

struct TableKey {
    int k, h, a;
    bool operator<(const TableKey &o) const { return std::tie(k, h, a) < std::tie(o.k, o.h, o.a); }
};

}  // namespace

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
    std::map<int, std::unique_ptr<Graph>> graphs;
    std::map<int, std::unique_ptr<Template>> tmpls;
    int next_graph = 1, next_tmpl = 1;
    std::map<TableKey, DevMem> split_tabs, drop_tabs;
    DevMem arena, colbuf, xbuf, npre;
    // options
    int64_t max_batch = SC_MAX_BATCH, fused = 1, use_graph = 0, tile_cols = 0, segment = 0;
    int64_t fuse_max_cols = 512, reorder = 1;
    // tracing
    bool prof = false;
    struct Rec { const char *name; hipEvent_t a, b; double bytes, updates; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
};

namespace {

int fail(sc_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, SC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

int dev_alloc(sc_ctx *c, DevMem &m, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->alloc) {
        p = c->alloc(bytes, (void *)c->stream, c->user);
        if (!p) return fail(c, SC_ENOMEM, "allocator hook returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, SC_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    m.p = p;
    m.bytes = bytes;
    return SC_OK;
}

void dev_free(sc_ctx *c, DevMem &m) {
    if (!m.p) return;
    if (c->free_fn) c->free_fn(m.p, m.bytes, (void *)c->stream, c->user);
    else (void)hipFree(m.p);
    m.p = nullptr;
    m.bytes = 0;
}

// Grows `m` to at least `bytes` (contents are not preserved).
int ensure(sc_ctx *c, DevMem &m, size_t bytes) {
    if (m.p && m.bytes >= bytes) return SC_OK;
    if (m.p) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, SC_EDEVICE, "stream sync failed");
        dev_free(c, m);
    }
    return dev_alloc(c, m, bytes);
}

int upload(sc_ctx *c, DevMem &m, const void *host, size_t bytes) {
    int rc = dev_alloc(c, m, bytes);
    if (rc) return rc;
    if (bytes) HIPCHK(c, hipMemcpyAsync(m.p, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SC_OK;
}

int default_segment(const sc_ctx *c) { return c->segment > 0 ? (int)c->segment : 256; }
int default_tile(const sc_ctx *c) { return c->tile_cols > 0 ? (int)c->tile_cols : 128; }

// Degree bins (see kernels.h): light rows, wide items (split rows first), and
// the compact slot of every split row for precomputed neighbour sums.
int rebin(sc_ctx *c, Graph &g, int seg) {
    if (g.seg == seg && g.slot.p) return SC_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dev_free(c, g.light); dev_free(c, g.wide); dev_free(c, g.split_rows); dev_free(c, g.slot);
    dev_free(c, g.tasks);
    std::vector<int32_t> light, split_rows, slot(std::max<int64_t>(g.n_rows, 1), -1);
    std::vector<int2> split_items, wide_items, split_tasks, tasks;
    for (int64_t v = 0; v < g.n_rows; ++v) {
        const int64_t d = g.deg_host[v];
        if (d <= kern::kLightMax) light.push_back((int32_t)v);
        else if (d <= seg) wide_items.push_back(make_int2((int)v, 0));
        if (d <= seg) {
            tasks.push_back(make_int2((int)v, 0));
        } else {
            slot[v] = (int32_t)split_rows.size();
            split_rows.push_back((int32_t)v);
            for (int64_t s = 0; s * seg < d; ++s) {
                split_items.push_back(make_int2((int)v, (int)s));
                split_tasks.push_back(make_int2((int)v, (int)s));
            }
        }
    }
    g.n_light = (int64_t)light.size();
    g.n_split = (int64_t)split_rows.size();
    g.n_split_items = (int64_t)split_items.size();
    std::vector<int2> items = split_items;
    items.insert(items.end(), wide_items.begin(), wide_items.end());
    g.n_wide = (int64_t)items.size();
    g.n_split_tasks = (int64_t)split_tasks.size();
    split_tasks.insert(split_tasks.end(), tasks.begin(), tasks.end());
    g.n_tasks = (int64_t)split_tasks.size();
    int rc;
    if ((rc = upload(c, g.light, light.data(), light.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, g.wide, items.data(), items.size() * sizeof(int2)))) return rc;
    if ((rc = upload(c, g.split_rows, split_rows.data(), split_rows.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, g.slot, slot.data(), slot.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, g.tasks, split_tasks.data(), split_tasks.size() * sizeof(int2)))) return rc;
    g.seg = seg;
    return SC_OK;
}

kern::GraphBins bins_of(const Graph &g) {
    kern::GraphBins b;
    b.n = g.n_rows; b.nnz = g.nnz;
    b.row_ptr = (const int64_t *)g.rp.p;
    b.col_idx = (const int32_t *)g.ci.p;
    b.light_rows = (const int32_t *)g.light.p; b.n_light = g.n_light;
    b.wide_items = (const int2 *)g.wide.p; b.n_wide = g.n_wide;
    b.split_rows = (const int32_t *)g.split_rows.p; b.n_split = g.n_split;
    b.n_split_items = g.n_split_items;
    b.slot = (const int32_t *)g.slot.p;
    b.tasks = (const int2 *)g.tasks.p; b.n_tasks = g.n_tasks; b.n_split_tasks = g.n_split_tasks;
    b.seg = g.seg;
    return b;
}

int get_split(sc_ctx *c, int k, int h, int a, const uint32_t **out) {
    TableKey key{k, h, a};
    auto it = c->split_tabs.find(key);
    if (it == c->split_tabs.end()) {
        std::vector<uint32_t> tab = split_table(k, h, a);
        DevMem m;
        int rc = upload(c, m, tab.data(), tab.size() * sizeof(uint32_t));
        if (rc) return rc;
        it = c->split_tabs.emplace(key, m).first;
    }
    *out = (const uint32_t *)it->second.p;
    return SC_OK;
}

int get_drop(sc_ctx *c, int k, int h, const int16_t **out) {
    TableKey key{k, h, 1};
    auto it = c->drop_tabs.find(key);
    if (it == c->drop_tabs.end()) {
        std::vector<int16_t> tab = drop_table(k, h);
        DevMem m;
        int rc = upload(c, m, tab.data(), tab.size() * sizeof(int16_t));
        if (rc) return rc;
        it = c->drop_tabs.emplace(key, m).first;
    }
    *out = (const int16_t *)it->second.p;
    return SC_OK;
}

ExecOpts exec_opts(const sc_ctx *c) {
    ExecOpts o;
    o.fuse = c->fused != 0;
    o.fuse_max_cols = (int)c->fuse_max_cols;
    return o;
}

int make_plan(sc_ctx *c, const Graph &g, const Template &T, int k, int batch, Plan &P) {
    std::string err;
    bool ok;
    const ExecOpts o = exec_opts(c);
    const int64_t rows = std::max<int64_t>(g.n_rows, 1);
    if (T.explicit_plan)
        ok = build_plan(T.t, T.root, T.child_ptr, T.child_idx, k, rows, g.nnz, batch, o, P, err);
    else
        ok = choose_plan(T.t, T.edges.data(), T.root, k, rows, g.nnz, batch, o, P, err);
    if (!ok) return fail(c, SC_EINVAL, "planning failed: %s", err.c_str());
    return SC_OK;
}

// Largest batch <= want whose arena fits the budget.
int pick_batch(sc_ctx *c, const Graph &g, const Template &T, int k, int want, Plan &P) {
    want = std::max(1, std::min<int>(want, (int)std::min<int64_t>(c->max_batch, SC_MAX_BATCH)));
    for (int b = want; b >= 1; --b) {
        int rc = make_plan(c, g, T, k, b, P);
        if (rc) return rc;
        uint64_t need = P.arena_bytes + (uint64_t)g.n_rows * b;
        if (need <= c->budget) return SC_OK;
        if (b == 1)
            return fail(c, SC_ENOMEM, "one colouring needs %.3f GB of tables, budget is %.3f GB",
                        need / 1e9, c->budget / 1e9);
    }
    return SC_OK;
}

// ---------------------------------------------------------------- tracing

hipEvent_t next_event(sc_ctx *c) {
    if (c->events_used == c->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->event_pool.push_back(e);
    }
    return c->event_pool[c->events_used++];
}

struct ProfScope {
    sc_ctx *c;
    hipStream_t st;
    const char *name;
    double bytes, updates;
    hipEvent_t a = nullptr;
    ProfScope(sc_ctx *c_, hipStream_t st_, const char *n, double by, double up)
        : c(c_), st(st_), name(n), bytes(by), updates(up) {
        if (c->prof && (a = next_event(c))) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = next_event(c);
        if (!b) return;
        (void)hipEventRecord(b, st);
        c->recs.push_back({name, a, b, bytes, updates});
    }
};

// One pass: colourings first..first+P.batch-1 folded into the table columns.
int run_pass(sc_ctx *c, Graph &g, const Plan &P, uint64_t first, hipStream_t st,
             uint64_t *counts, uint8_t *flags_out) {
    const int B = P.batch, k = P.k;
    const int64_t n = g.n_rows;            // table rows
    const double dn = (double)n, dnnz = (double)g.nnz;
    int rc;
    if (P.steps.empty() || n == 0) {       // t == 1: every vertex is a map; no edges: no map
        for (int r = 0; r < B; ++r) { counts[r] = P.steps.empty() ? (uint64_t)g.n : 0; flags_out[r] = 0; }
        return SC_OK;
    }
    if ((rc = rebin(c, g, default_segment(c)))) return rc;
    if ((rc = ensure(c, c->arena, P.arena_bytes))) return rc;
    if ((rc = ensure(c, c->colbuf, (size_t)n * B))) return rc;
    if ((rc = ensure(c, c->xbuf, (SC_MAX_BATCH + 1) * sizeof(uint64_t)))) return rc;
    size_t npre_words = 0;
    for (const Step &s : P.steps)
        if (s.mode == kStepFusedHist || s.mode == kStepFusedGather)
            npre_words = std::max(npre_words, (size_t)g.n_split * binom(k, s.p) * B);
    if (npre_words && (rc = ensure(c, c->npre, npre_words * 8))) return rc;
    auto *X = (unsigned long long *)c->xbuf.p;
    auto *flags = X + SC_MAX_BATCH;
    auto *col = (uint8_t *)c->colbuf.p;
    auto *base = (uint8_t *)c->arena.p;
    auto *Npre = (uint64_t *)c->npre.p;
    auto buf = [&](int id) { return id < 0 ? (uint64_t *)nullptr : (uint64_t *)(base + P.bufs[id].offset); };
    const kern::GraphBins bins = bins_of(g);
    const double adj_bytes = 4.0 * dnnz + 8.0 * (dn + 1);
    double split_nnz = 0;
    if (g.n_split) for (int64_t v = 0; v < n; ++v) if (g.deg_host[v] > g.seg) split_nnz += (double)g.deg_host[v];

    HIPCHK(c, kern::launch_zero_u64((uint64_t *)X, SC_MAX_BATCH + 1, st));
    {
        ProfScope ps(c, st, "color", dn * B, 0);
        HIPCHK(c, kern::launch_color(c->seed, first, n, B, k, (const int32_t *)g.perm.p, col, st));
    }
    const Step *last = nullptr;
    for (const Step &s : P.steps) {
        const int Wa = (int)binom(k, s.a), Wp = (int)binom(k, s.p), Wh = (int)binom(k, s.h);
        const int64_t Lp = (int64_t)Wp * B;
        const double La = (double)Wa * B, Ls = (double)Wh * B, dLp = (double)Lp;
        const int nsplit = (int)binom(s.h, s.a);
        uint64_t *N = buf(s.buf_n);
        uint64_t *S = buf(s.buf_s);
        const uint64_t *Pp = buf(s.buf_p), *A = buf(s.buf_a);
        const uint32_t *split = nullptr;
        const int16_t *drop = nullptr;
        if (s.a > 1) { if ((rc = get_split(c, k, s.h, s.a, &split))) return rc; }
        else { if ((rc = get_drop(c, k, s.h, &drop))) return rc; }
        const double ema_upd = s.a > 1 ? dn * Ls * nsplit : dn * Ls;
        const double ema_bytes = 8.0 * dn * ((s.a > 1 ? La : 0) + Ls) + (s.a == 1 ? dn * B : 0);
        const double sp_upd = dnnz * dLp;
        switch (s.mode) {
        case kStepFusedHist: {
            if (g.n_split) {
                ProfScope ps(c, st, "hist_split", 4.0 * split_nnz + 8.0 * g.n_split * dLp, split_nnz * dLp);
                HIPCHK(c, kern::launch_hist_split(bins, col, Npre, B, k, st));
            }
            ProfScope ps(c, st, "row_hist", adj_bytes + dn * B + ema_bytes, sp_upd + ema_upd);
            HIPCHK(c, kern::launch_row(kern::kModeHist, bins, col, nullptr, Npre, A, S, B, k, s.a,
                                       Wa, Wp, Wh, nsplit, split, drop, flags, st));
            break;
        }
        case kStepFusedGather: {
            if (g.n_split) {
                HIPCHK(c, kern::launch_zero_split_rows(bins, true, Npre, Lp, st));
                ProfScope ps(c, st, "spmm_split", 4.0 * split_nnz + 16.0 * g.n_split * dLp, split_nnz * dLp);
                HIPCHK(c, kern::launch_spmm_split(bins, Pp, Npre, Lp, B, default_tile(c), flags, st));
            }
            ProfScope ps(c, st, "row_gather", adj_bytes + 8.0 * dn * dLp + ema_bytes, sp_upd + ema_upd);
            HIPCHK(c, kern::launch_row(kern::kModeGather, bins, col, Pp, Npre, A, S, B, k, s.a,
                                       Wa, Wp, Wh, nsplit, split, drop, flags, st));
            break;
        }
        default: {
            if (s.p == 1) {
                ProfScope ps(c, st, "hist", adj_bytes + dn * B + 8.0 * dn * dLp, sp_upd);
                HIPCHK(c, kern::launch_hist(bins, col, N, B, k, st));
            } else {
                HIPCHK(c, kern::launch_zero_split_rows(bins, false, N, Lp, st));
                ProfScope ps(c, st, "spmm", adj_bytes + 16.0 * dn * dLp, sp_upd);
                HIPCHK(c, kern::launch_spmm(bins, Pp, N, Lp, B, default_tile(c), flags, st));
            }
            if (s.mode == kStepStaged) {
                ProfScope ps(c, st, "row_staged", 8.0 * dn * dLp + ema_bytes, ema_upd);
                HIPCHK(c, kern::launch_row(kern::kModeStaged, bins, col, N, nullptr, A, S, B, k, s.a,
                                           Wa, Wp, Wh, nsplit, split, drop, flags, st));
            } else if (s.a == 1) {
                ProfScope ps(c, st, "select", 8.0 * dn * dLp + ema_bytes, ema_upd);
                HIPCHK(c, kern::launch_select(n, col, N, S, B, k, Wh, Wp, drop, st));
            } else {
                ProfScope ps(c, st, "ema", 8.0 * dn * dLp + ema_bytes, ema_upd);
                HIPCHK(c, kern::launch_ema(n, A, N, S, B, Wa, Wp, Wh, nsplit, split, flags, st));
            }
        }
        }
        last = &s;
    }
    {
        const int W = (int)binom(k, last->h);
        ProfScope ps(c, st, "reduce", 8.0 * dn * W * B, 0);
        HIPCHK(c, kern::launch_reduce(n, buf(last->buf_s), W, B, X, flags, st));
    }
    uint64_t host[SC_MAX_BATCH + 1];
    HIPCHK(c, hipMemcpyAsync(host, X, sizeof host, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int r = 0; r < B; ++r) {
        counts[r] = host[r];
        flags_out[r] = (uint8_t)((host[SC_MAX_BATCH] >> r) & 1);
    }
    return SC_OK;
}

double colorful_probability(int k, int t) {
    double p = 1.0;
    for (int i = 0; i < t; ++i) p *= (double)(k - i) / (double)k;
    return p;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *sc_version(void) { return "libsc 0.1 (gfx950)"; }

const char *sc_last_error(const sc_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int sc_create(int device, sc_alloc_fn alloc, sc_free_fn free_fn, void *user, uint64_t budget,
              sc_ctx **out) {
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return SC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { (void)hipGetLastError(); return SC_EDEVICE; }
    if (device < 0 || device >= ndev) return SC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SC_EDEVICE;
    auto *c = new sc_ctx();
    c->device = device;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return SC_EDEVICE; }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipStreamDestroy(c->stream); delete c; return SC_EDEVICE; }
    c->budget = budget ? budget : (uint64_t)(0.9 * (double)fr);
    *out = c;
    return SC_OK;
}

int sc_destroy(sc_ctx *c) {
    if (!c) return SC_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->graphs) {
        Graph &g = *kv.second;
        dev_free(c, g.rp); dev_free(c, g.ci); dev_free(c, g.light); dev_free(c, g.wide);
        dev_free(c, g.split_rows); dev_free(c, g.slot); dev_free(c, g.perm); dev_free(c, g.tasks);
    }
    for (auto &kv : c->split_tabs) dev_free(c, kv.second);
    for (auto &kv : c->drop_tabs) dev_free(c, kv.second);
    dev_free(c, c->arena); dev_free(c, c->colbuf); dev_free(c, c->xbuf); dev_free(c, c->npre);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return SC_OK;
}

int sc_load_graph_csr(sc_ctx *c, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci,
                      int32_t *graph_id) {
    if (!c) return SC_EINVAL;
    if (!rp || !graph_id || (nnz > 0 && !ci)) return fail(c, SC_EINVAL, "NULL argument");
    if (n < 1 || n >= (int64_t)1 << 31) return fail(c, SC_EINVAL, "n must be in [1, 2^31)");
    if (nnz < 0 || rp[0] != 0 || rp[n] != nnz) return fail(c, SC_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
    for (int64_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) return fail(c, SC_EINVAL, "row_ptr decreases at row %lld", (long long)v);
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t j = ci[e];
            if (j < 0 || j >= n) return fail(c, SC_EINVAL, "column %d out of range in row %lld", j, (long long)v);
            if (j == v) return fail(c, SC_EINVAL, "self-loop at vertex %lld", (long long)v);
            if (e > rp[v] && ci[e - 1] >= j) return fail(c, SC_EINVAL, "row %lld is not strictly increasing", (long long)v);
        }
    }
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t j = ci[e];
            if (!std::binary_search(ci + rp[j], ci + rp[j + 1], (int32_t)v))
                return fail(c, SC_EINVAL, "adjacency is not symmetric: (%lld,%d) without (%d,%lld)",
                            (long long)v, j, j, (long long)v);
        }
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    auto g = std::make_unique<Graph>();
    g->n = n;
    g->nnz = nnz;
    g->deg_host.resize(n);
    int rc;
    if (c->reorder) {
        // Relabel by descending degree: the rows that neighbour sums gather most
        // often become one contiguous region.  Colours are still drawn from the
        // original ids (perm), so every count is unchanged.
        std::vector<int32_t> perm(n), inv(n);
        for (int64_t v = 0; v < n; ++v) perm[v] = (int32_t)v;
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) {
            return rp[x + 1] - rp[x] > rp[y + 1] - rp[y];
        });
        for (int64_t v = 0; v < n; ++v) inv[perm[v]] = (int32_t)v;
        std::vector<int64_t> nrp(n + 1, 0);
        for (int64_t v = 0; v < n; ++v) nrp[v + 1] = nrp[v] + (rp[perm[v] + 1] - rp[perm[v]]);
        std::vector<int32_t> nci((size_t)std::max<int64_t>(nnz, 1));
        for (int64_t v = 0; v < n; ++v) {
            const int32_t u = perm[v];
            int32_t *dst = nci.data() + nrp[v];
            for (int64_t e = rp[u]; e < rp[u + 1]; ++e) *dst++ = inv[ci[e]];
            std::sort(nci.data() + nrp[v], nci.data() + nrp[v + 1]);
        }
        for (int64_t v = 0; v < n; ++v) g->deg_host[v] = nrp[v + 1] - nrp[v];
        g->n_rows = 0;
        while (g->n_rows < n && g->deg_host[g->n_rows] > 0) ++g->n_rows;
        if ((rc = upload(c, g->rp, nrp.data(), (size_t)(n + 1) * sizeof(int64_t)))) return rc;
        if ((rc = upload(c, g->ci, nci.data(), (size_t)nnz * sizeof(int32_t)))) { dev_free(c, g->rp); return rc; }
        if ((rc = upload(c, g->perm, perm.data(), (size_t)n * sizeof(int32_t)))) {
            dev_free(c, g->rp); dev_free(c, g->ci); return rc;
        }
    } else {
        for (int64_t v = 0; v < n; ++v) g->deg_host[v] = rp[v + 1] - rp[v];
        g->n_rows = n;
        if ((rc = upload(c, g->rp, rp, (size_t)(n + 1) * sizeof(int64_t)))) return rc;
        if ((rc = upload(c, g->ci, ci, (size_t)nnz * sizeof(int32_t)))) { dev_free(c, g->rp); return rc; }
    }
    if ((rc = rebin(c, *g, default_segment(c)))) {
        dev_free(c, g->rp); dev_free(c, g->ci); dev_free(c, g->perm); return rc;
    }
    *graph_id = c->next_graph++;
    c->graphs[*graph_id] = std::move(g);
    return SC_OK;
}

int sc_unload_graph(sc_ctx *c, int32_t id) {
    if (!c) return SC_EINVAL;
    auto it = c->graphs.find(id);
    if (it == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", id);
    (void)hipStreamSynchronize(c->stream);
    Graph &g = *it->second;
    dev_free(c, g.rp); dev_free(c, g.ci); dev_free(c, g.light); dev_free(c, g.wide);
    dev_free(c, g.split_rows); dev_free(c, g.slot); dev_free(c, g.perm); dev_free(c, g.tasks);
    c->graphs.erase(it);
    return SC_OK;
}

static double aut_of(int t, const std::vector<int32_t> &edges) {
    std::vector<std::pair<int, int>> e;
    for (int i = 0; i + 1 < (int)edges.size(); i += 2) e.emplace_back(edges[i], edges[i + 1]);
    return tree_automorphisms(t, e);
}

int sc_load_template(sc_ctx *c, int32_t t, const int32_t *edges, int32_t root, int32_t *tmpl_id) {
    if (!c) return SC_EINVAL;
    if (!tmpl_id) return fail(c, SC_EINVAL, "NULL argument");
    std::string m = check_tree(t, edges);
    if (!m.empty()) return fail(c, SC_EINVAL, "%s", m.c_str());
    if (root < -1 || root >= t) return fail(c, SC_EINVAL, "root out of range");
    auto T = std::make_unique<Template>();
    T->t = t;
    T->edges.assign(edges, edges + 2 * (t - 1));
    T->root = root;
    T->aut = aut_of(t, T->edges);
    *tmpl_id = c->next_tmpl++;
    c->tmpls[*tmpl_id] = std::move(T);
    return SC_OK;
}

int sc_load_template_plan(sc_ctx *c, int32_t t, int32_t root, const int32_t *child_ptr,
                          const int32_t *child_idx, int32_t *tmpl_id) {
    if (!c) return SC_EINVAL;
    if (!child_ptr || !tmpl_id || (t > 1 && !child_idx)) return fail(c, SC_EINVAL, "NULL argument");
    if (t < 1 || t > SC_MAX_T) return fail(c, SC_EINVAL, "template size must be in [1, 16]");
    auto T = std::make_unique<Template>();
    T->t = t;
    T->root = root;
    T->explicit_plan = true;
    T->child_ptr.assign(child_ptr, child_ptr + t + 1);
    T->child_idx.assign(child_idx, child_idx + (t - 1));
    Plan probe;
    std::string err;
    if (!build_plan(t, root, T->child_ptr, T->child_idx, t, 1, 0, 1, ExecOpts(), probe, err))
        return fail(c, SC_EINVAL, "%s", err.c_str());
    for (int u = 0; u < t; ++u)
        for (int e = child_ptr[u]; e < child_ptr[u + 1]; ++e) {
            T->edges.push_back(u);
            T->edges.push_back(child_idx[e]);
        }
    T->aut = aut_of(t, T->edges);
    *tmpl_id = c->next_tmpl++;
    c->tmpls[*tmpl_id] = std::move(T);
    return SC_OK;
}

int sc_set_colors(sc_ctx *c, int32_t k, uint64_t seed) {
    if (!c) return SC_EINVAL;
    if (k < 1 || k > SC_MAX_K) return fail(c, SC_EINVAL, "k must be in [1, %d]", SC_MAX_K);
    c->k = k;
    c->seed = seed;
    return SC_OK;
}

int sc_set_option(sc_ctx *c, int32_t opt, int64_t v) {
    if (!c) return SC_EINVAL;
    switch (opt) {
    case SC_OPT_MAX_BATCH:
        if (v < 1 || v > SC_MAX_BATCH) return fail(c, SC_EINVAL, "max batch must be in [1, %d]", SC_MAX_BATCH);
        c->max_batch = v; return SC_OK;
    case SC_OPT_FUSED: c->fused = v != 0; return SC_OK;
    case SC_OPT_GRAPH: c->use_graph = v != 0; return SC_OK;
    case SC_OPT_TILE_COLS:
        if (v != 0 && v != 8 && v != 16 && v != 32 && v != 64 && v != 128 && v != 256)
            return fail(c, SC_EINVAL, "tile columns must be 0, 8, 16, 32, 64, 128 or 256");
        c->tile_cols = v; return SC_OK;
    case SC_OPT_SEGMENT:
        if (v < 0 || v > (1 << 24)) return fail(c, SC_EINVAL, "segment must be in [0, 2^24]");
        if (v > 0 && v <= kern::kLightMax) return fail(c, SC_EINVAL, "segment must exceed %d", kern::kLightMax);
        c->segment = v; return SC_OK;
    case SC_OPT_FUSE_MAX_COLS:
        if (v < 64 || v > 2048) return fail(c, SC_EINVAL, "fuse max columns must be in [64, 2048]");
        c->fuse_max_cols = v; return SC_OK;
    case SC_OPT_REORDER: c->reorder = v != 0; return SC_OK;
    default: return fail(c, SC_EINVAL, "unknown option %d", opt);
    }
}

int sc_get_option(sc_ctx *c, int32_t opt, int64_t *v) {
    if (!c || !v) return SC_EINVAL;
    switch (opt) {
    case SC_OPT_MAX_BATCH: *v = c->max_batch; return SC_OK;
    case SC_OPT_FUSED: *v = c->fused; return SC_OK;
    case SC_OPT_GRAPH: *v = c->use_graph; return SC_OK;
    case SC_OPT_TILE_COLS: *v = default_tile(c); return SC_OK;
    case SC_OPT_SEGMENT: *v = default_segment(c); return SC_OK;
    case SC_OPT_FUSE_MAX_COLS: *v = c->fuse_max_cols; return SC_OK;
    case SC_OPT_REORDER: *v = c->reorder; return SC_OK;
    default: return fail(c, SC_EINVAL, "unknown option %d", opt);
    }
}

int sc_plan_template(int32_t t, const int32_t *edges, int32_t root, int32_t k, int64_t n,
                     int64_t nnz, int32_t batch, sc_plan_info_t *out) {
    if (!out || batch < 1 || batch > SC_MAX_BATCH || n < 1 || nnz < 0) return SC_EINVAL;
    Plan P;
    std::string err;
    if (!choose_plan(t, edges, root, k, n, nnz, batch, ExecOpts(), P, err)) return SC_EINVAL;
    std::vector<int32_t> e(edges ? edges : (const int32_t *)nullptr, edges ? edges + 2 * (t - 1) : nullptr);
    fill_plan_info(P, aut_of(t, e), out);
    return SC_OK;
}

int sc_plan_info(sc_ctx *c, int32_t gid, int32_t tid, int32_t n_colorings, sc_plan_info_t *out) {
    if (!c) return SC_EINVAL;
    if (!out) return fail(c, SC_EINVAL, "NULL argument");
    auto gi = c->graphs.find(gid);
    if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", gid);
    auto ti = c->tmpls.find(tid);
    if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", tid);
    if (c->k < ti->second->t) return fail(c, SC_EINVAL, "k=%d < t=%d (call sc_set_colors)", c->k, ti->second->t);
    Plan P;
    int rc = pick_batch(c, *gi->second, *ti->second, c->k, std::max(1, n_colorings), P);
    if (rc) return rc;
    fill_plan_info(P, ti->second->aut, out);
    return SC_OK;
}

int64_t sc_colorset_rank(uint32_t mask) { return colorset_rank(mask); }

int32_t sc_color_of(uint64_t seed, uint64_t coloring, uint64_t v, int32_t k) {
    uint64_t idx = (coloring << 40) + v;
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (int32_t)(((unsigned __int128)z * (uint64_t)(uint32_t)k) >> 64);
}

int sc_run(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, int32_t ncol, void *stream,
           uint64_t *counts, uint8_t *overflow, double *est_maps, double *est_copies) {
    if (!c) return SC_EINVAL;
    if (ncol < 0) return fail(c, SC_EINVAL, "n_colorings < 0");
    if (ncol > 0 && (!counts || !overflow)) return fail(c, SC_EINVAL, "NULL output");
    auto gi = c->graphs.find(gid);
    if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", gid);
    auto ti = c->tmpls.find(tid);
    if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", tid);
    Graph &g = *gi->second;
    const Template &T = *ti->second;
    const int k = c->k;
    if (k < T.t) return fail(c, SC_EINVAL, "k=%d < t=%d (call sc_set_colors)", k, T.t);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    int rc;
    Plan P;
    int done = 0;
    bool any_ovf = false;
    double sum = 0.0;
    while (done < ncol) {
        if ((rc = pick_batch(c, g, T, k, ncol - done, P))) return rc;
        if ((rc = run_pass(c, g, P, first + (uint64_t)done, st, counts + done, overflow + done))) return rc;
        for (int r = 0; r < P.batch; ++r) {
            any_ovf |= overflow[done + r] != 0;
            sum += (double)counts[done + r];
        }
        done += P.batch;
    }
    double maps = NAN, copies = NAN;
    if (ncol > 0 && !any_ovf) {
        maps = sum / ncol / colorful_probability(k, T.t);
        copies = maps / T.aut;
    }
    if (est_maps) *est_maps = maps;
    if (est_copies) *est_copies = copies;
    return SC_OK;
}

int sc_profile(sc_ctx *c, int32_t enable) {
    if (!c) return SC_EINVAL;
    if (enable) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->recs.clear();
        c->events_used = 0;
    }
    c->prof = enable != 0;
    return SC_OK;
}

int sc_profile_read(sc_ctx *c, sc_kernel_stat_t *out, int32_t cap, int32_t *n_out) {
    if (!c) return SC_EINVAL;
    if (!n_out || (cap > 0 && !out)) return fail(c, SC_EINVAL, "NULL argument");
    std::vector<sc_kernel_stat_t> agg;
    for (auto &r : c->recs) {
        HIPCHK(c, hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
        sc_kernel_stat_t *hit = nullptr;
        for (auto &a : agg) if (!strcmp(a.name, r.name)) hit = &a;
        if (!hit) {
            agg.emplace_back();
            hit = &agg.back();
            std::memset(hit, 0, sizeof *hit);
            std::snprintf(hit->name, sizeof hit->name, "%s", r.name);
        }
        hit->launches += 1;
        hit->total_ms += ms;
        hit->alg_bytes += r.bytes;
        hit->updates += r.updates;
    }
    *n_out = (int32_t)agg.size();
    for (int32_t i = 0; i < cap && i < (int32_t)agg.size(); ++i) out[i] = agg[i];
    return SC_OK;
}

}  // extern "C"
