// libsc runtime: contexts, device memory, resident graphs and templates,
// options, tracing, planning queries, and the C ABI for all of them.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "rt.h"

namespace sc {

int fail(sc_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

int dev_alloc(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 256;
    if (!st) st = c->stream;
    void *p = c->alloc(bytes, (void *)st, c->user);
    if (!p) return fail(c, SC_ENOMEM, "the allocator hook returned NULL for %zu bytes", bytes);
    m.p = p;
    m.bytes = bytes;
    m.stream = st;
    return SC_OK;
}

void dev_free(sc_ctx *c, DevMem &m) {
    if (!m.p) return;
    c->free_fn(m.p, m.bytes, (void *)m.stream, c->user);
    m.p = nullptr;
    m.bytes = 0;
    m.stream = nullptr;
}

int ensure(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st, uint64_t *gen) {
    if (m.p && m.bytes >= bytes) return SC_OK;
    if (m.p) {
        HIPCHK(c, hipStreamSynchronize(st));
        dev_free(c, m);
    }
    if (gen) ++*gen;
    return dev_alloc(c, m, bytes, st);
}

int upload(sc_ctx *c, DevMem &m, const void *host, size_t bytes) {
    int rc = dev_alloc(c, m, bytes);
    if (rc) return rc;
    if (bytes) HIPCHK(c, hipMemcpyAsync(m.p, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SC_OK;
}

int host_staging(sc_ctx *c, size_t words) {
    if (c->host_out && c->host_out_words >= words) return SC_OK;
    if (c->host_out) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        (void)hipHostFree(c->host_out);
        c->host_out = nullptr;
        c->host_out_words = 0;
    }
    void *p = nullptr;
    HIPCHK(c, hipHostMalloc(&p, words * sizeof(uint64_t), hipHostMallocDefault));
    c->host_out = (uint64_t *)p;
    c->host_out_words = words;
    return SC_OK;
}

int default_segment(const sc_ctx *c) { return c->segment > 0 ? (int)c->segment : 512; }

int plan_segment(const sc_ctx *c, const Plan &P) { return P.opts.seg > 0 ? P.opts.seg : default_segment(c); }

// Rows with more than `seg` neighbours ("split rows"): their (row, segment)
// items and the compact slot of every split row for precomputed neighbour sums.
// Bins of earlier segment sizes are kept, so switching back costs nothing.
int rebin(sc_ctx *c, Graph &g, int seg, bool allocate) {
    if (g.seg == seg && g.slot.p) return SC_OK;
    auto it = g.saved_bins.find(seg);
    if (it == g.saved_bins.end() && !allocate)
        return fail(c, SC_ESTATE, "graph has no heavy-row bins for segment size %d", seg);
    if (g.busy && it == g.saved_bins.end())
        return fail(c, SC_ESTATE, "segment size cannot change while the serving loop uses the graph");
    if (g.slot.p) {
        Graph::SavedBins &sv = g.saved_bins[g.seg];
        sv.split_rows = g.split_rows; sv.split_items = g.split_items; sv.slot = g.slot;
        sv.n_split = g.n_split; sv.n_split_items = g.n_split_items; sv.split_nnz = g.split_nnz;
        g.split_rows = g.split_items = g.slot = DevMem{};
    }
    it = g.saved_bins.find(seg);
    if (it != g.saved_bins.end()) {
        const Graph::SavedBins &sv = it->second;
        g.split_rows = sv.split_rows; g.split_items = sv.split_items; g.slot = sv.slot;
        g.n_split = sv.n_split; g.n_split_items = sv.n_split_items; g.split_nnz = sv.split_nnz;
        g.saved_bins.erase(it);
        g.seg = seg;
        return SC_OK;
    }
    std::vector<int32_t> split_rows, slot(std::max<int64_t>(g.n_rows, 1), -1);
    std::vector<int2> items;
    g.split_nnz = 0;
    for (int64_t v = 0; v < g.n_rows; ++v) {
        const int64_t d = g.deg_host[v];
        if (d <= seg) continue;
        slot[v] = (int32_t)split_rows.size();
        split_rows.push_back((int32_t)v);
        g.split_nnz += (double)d;
        for (int64_t s = 0; s * seg < d; ++s) items.push_back(make_int2((int)v, (int)s));
    }
    g.n_split = (int64_t)split_rows.size();
    g.n_split_items = (int64_t)items.size();
    int rc;
    if ((rc = upload(c, g.split_rows, split_rows.data(), split_rows.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, g.split_items, items.data(), items.size() * sizeof(int2)))) return rc;
    if ((rc = upload(c, g.slot, slot.data(), slot.size() * sizeof(int32_t)))) return rc;
    g.seg = seg;
    return SC_OK;
}

kern::GraphBins bins_of(const Graph &g) {
    kern::GraphBins b;
    b.n = g.n_rows; b.nnz = g.nnz;
    b.row_ptr = (const int64_t *)g.rp.p;
    b.col_idx = (const int32_t *)g.ci.p;
    b.split_rows = (const int32_t *)g.split_rows.p; b.n_split = g.n_split;
    b.split_items = (const int2 *)g.split_items.p; b.n_split_items = g.n_split_items;
    b.slot = (const int32_t *)g.slot.p;
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

int get_unrank(sc_ctx *c, int k1, int sz, const uint16_t **out) {
    TableKey key{k1, sz, 0};
    auto it = c->unrank_tabs.find(key);
    if (it == c->unrank_tabs.end()) {
        std::vector<uint16_t> tab = unrank_table(k1, sz);
        DevMem m;
        int rc = upload(c, m, tab.data(), tab.size() * sizeof(uint16_t));
        if (rc) return rc;
        it = c->unrank_tabs.emplace(key, m).first;
    }
    *out = (const uint16_t *)it->second.p;
    return SC_OK;
}

int get_rank(sc_ctx *c, int k1, const uint16_t **out) {
    TableKey key{k1, 0, 0};
    auto it = c->rank_tabs.find(key);
    if (it == c->rank_tabs.end()) {
        std::vector<uint16_t> tab = rank_table(k1);
        DevMem m;
        int rc = upload(c, m, tab.data(), tab.size() * sizeof(uint16_t));
        if (rc) return rc;
        it = c->rank_tabs.emplace(key, m).first;
    }
    *out = (const uint16_t *)it->second.p;
    return SC_OK;
}

ExecOpts exec_opts(const sc_ctx *c, int gid, int tid, int k, int batch) {
    ExecOpts o;
    o.interleave = (int)c->interleave;
    if (c->lds_max > 0) o.lds_max = (int)c->lds_max;
    if (c->wave_row_max >= 0) o.wave_row_max = (int)c->wave_row_max;
    o.chain = (int)c->chain;
    auto it = c->tuned.find(TuneKey{gid, tid, k, batch});
    if (it != c->tuned.end()) {
        if (it->second.interleave > 0) o.interleave = it->second.interleave;
        if (it->second.lds_max > 0) o.lds_max = it->second.lds_max;
        if (it->second.seg > 0) o.seg = it->second.seg;
        if (it->second.wave_row_max >= 0) o.wave_row_max = it->second.wave_row_max;
    }
    return o;
}

int make_plan(sc_ctx *c, const Graph &g, const Template &T, const ExecOpts &o, int k, int batch,
              Plan &P) {
    std::string err;
    bool ok;
    const int64_t rows = std::max<int64_t>(g.n_rows, 1);
    if (T.explicit_plan)
        ok = build_plan(T.t, T.root, T.child_ptr, T.child_idx, k, rows, g.nnz, batch, o, P, err);
    else
        ok = choose_plan(T.t, T.edges.data(), T.root, k, rows, g.nnz, batch, o, P, err);
    if (!ok) return fail(c, SC_EINVAL, "planning failed: %s", err.c_str());
    // tables hold the non-isolated rows; the paper's counts run over every vertex
    lemma1_counts(P, g.n);
    return SC_OK;
}

uint64_t pass_bytes(const Graph &g, const Plan &P) {
    uint64_t npre = 0;
    for (const Step &s : P.steps)
        npre = std::max<uint64_t>(npre, (uint64_t)g.n_split * binom(P.k - 1, s.p) * P.batch * 8);
    return P.arena_bytes + npre + (uint64_t)g.n_rows * P.batch;
}

int pick_batch(sc_ctx *c, int gid, int tid, int k, int want, uint64_t budget, Plan &P) {
    auto gi = c->graphs.find(gid);
    if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", gid);
    auto ti = c->tmpls.find(tid);
    if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", tid);
    const Graph &g = *gi->second;
    const Template &T = *ti->second;
    if (k < T.t || k > SC_MAX_K) return fail(c, SC_EINVAL, "need t <= k <= 16 (t=%d, k=%d)", T.t, k);
    if (!budget) budget = c->budget;
    want = std::max(1, std::min<int>(want, (int)std::min<int64_t>(c->max_batch, SC_MAX_BATCH)));
    // `want`, then the multiples of 8 below it, then 4, 2, 1: batches with a
    // large power-of-two factor keep several colourings interleaved per plane
    for (int b = want; b >= 1;) {
        const ExecOpts o = exec_opts(c, gid, tid, k, b);
        int rc = make_plan(c, g, T, o, k, b, P);
        if (rc) return rc;
        if (pass_bytes(g, P) <= budget) return SC_OK;
        if (b > 8) b = b % 8 ? b - b % 8 : b - 8;
        else b = b > 4 ? 4 : b / 2;
    }
    return fail(c, SC_ENOMEM, "one colouring needs %.3f GB of device tables, the budget is %.3f GB",
                pass_bytes(g, P) / 1e9, budget / 1e9);
}

double colorful_probability(int k, int t) {
    double p = 1.0;
    for (int i = 0; i < t; ++i) p *= (double)(k - i) / (double)k;
    return p;
}

}  // namespace sc

using namespace sc;

namespace {

double aut_of(int t, const std::vector<int32_t> &edges) {
    std::vector<std::pair<int, int>> e;
    for (int i = 0; i + 1 < (int)edges.size(); i += 2) e.emplace_back(edges[i], edges[i + 1]);
    return tree_automorphisms(t, e);
}

void free_graph(sc_ctx *c, Graph &g) {
    dev_free(c, g.rp); dev_free(c, g.ci); dev_free(c, g.split_rows); dev_free(c, g.split_items);
    dev_free(c, g.slot); dev_free(c, g.perm);
    for (auto &kv : g.saved_bins) {
        dev_free(c, kv.second.split_rows); dev_free(c, kv.second.split_items); dev_free(c, kv.second.slot);
    }
    g.saved_bins.clear();
}

bool serving(const sc_ctx *c) { return c->serve != nullptr; }

}  // namespace

extern "C" {

const char *sc_version(void) { return "libsc 0.3 (gfx950)"; }

const char *sc_last_error(const sc_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int sc_create(int device, sc_alloc_fn alloc, sc_free_fn free_fn, void *user, uint64_t budget,
              sc_ctx **out) {
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if (!alloc || !free_fn) return SC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { (void)hipGetLastError(); return SC_EDEVICE; }
    if (device < 0 || device >= ndev) return SC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SC_EDEVICE;
    if (static_scratch_init(device) != SC_OK) return SC_EDEVICE;
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
    serve_shutdown(c);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
    drop_call_graphs(c);
    dev_free(c, c->call_desc); dev_free(c, c->call_x);
    for (auto &kv : c->graphs) free_graph(c, *kv.second);
    for (auto &kv : c->split_tabs) dev_free(c, kv.second);
    for (auto &kv : c->unrank_tabs) dev_free(c, kv.second);
    for (auto &kv : c->rank_tabs) dev_free(c, kv.second);
    PassBuffers &b = c->main;
    dev_free(c, b.arena); dev_free(c, b.colbuf); dev_free(c, b.xbuf); dev_free(c, b.npre); dev_free(c, b.desc);
    dev_free(c, c->wide_tab); dev_free(c, c->wide_x);
    if (c->host_out) (void)hipHostFree(c->host_out);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return SC_OK;
}

int sc_load_graph_csr(sc_ctx *c, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci,
                      int32_t *graph_id) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
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
        // Relabel by descending degree (1): the rows that neighbour sums gather
        // most often become one contiguous region and the isolated vertices the
        // tail; or in reverse Cuthill-McKee order (2), isolated vertices last.
        // Colours are still drawn from the caller's ids (perm), so every count
        // is unchanged.
        std::vector<int32_t> perm(n), inv(n);
        auto deg = [&](int32_t x) { return rp[x + 1] - rp[x]; };
        for (int64_t v = 0; v < n; ++v) perm[v] = (int32_t)v;
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
        if (c->reorder == 2) {
            // breadth-first from each component's lowest-degree vertex,
            // neighbours in ascending degree, then reversed
            std::vector<int32_t> order;
            order.reserve(n);
            std::vector<uint8_t> seen(n, 0);
            std::vector<int32_t> nb;
            for (int64_t i = n - 1; i >= 0; --i) {
                const int32_t s0 = perm[i];
                if (seen[s0] || deg(s0) == 0) continue;
                size_t head = order.size();
                order.push_back(s0);
                seen[s0] = 1;
                while (head < order.size()) {
                    const int32_t u = order[head++];
                    nb.assign(ci + rp[u], ci + rp[u + 1]);
                    std::stable_sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg(x) < deg(y); });
                    for (int32_t w : nb)
                        if (!seen[w]) { seen[w] = 1; order.push_back(w); }
                }
            }
            std::reverse(order.begin(), order.end());
            for (int64_t v = 0; v < n; ++v)
                if (deg((int32_t)v) == 0) order.push_back((int32_t)v);
            perm.swap(order);
        }
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
        if ((rc = upload(c, g->ci, nci.data(), (size_t)nnz * sizeof(int32_t)))) { free_graph(c, *g); return rc; }
        if ((rc = upload(c, g->perm, perm.data(), (size_t)n * sizeof(int32_t)))) { free_graph(c, *g); return rc; }
    } else {
        for (int64_t v = 0; v < n; ++v) g->deg_host[v] = rp[v + 1] - rp[v];
        g->n_rows = n;
        if ((rc = upload(c, g->rp, rp, (size_t)(n + 1) * sizeof(int64_t)))) return rc;
        if ((rc = upload(c, g->ci, ci, (size_t)nnz * sizeof(int32_t)))) { free_graph(c, *g); return rc; }
    }
    for (int64_t v = 0; v < n; ++v) g->max_deg = std::max(g->max_deg, g->deg_host[v]);
    if ((rc = rebin(c, *g, default_segment(c)))) { free_graph(c, *g); return rc; }
    *graph_id = c->next_graph++;
    c->graphs[*graph_id] = std::move(g);
    return SC_OK;
}

int sc_unload_graph(sc_ctx *c, int32_t id) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    auto it = c->graphs.find(id);
    if (it == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", id);
    if (it->second->busy) return fail(c, SC_EBUSY, "graph %d has serving passes in flight", id);
    (void)hipDeviceSynchronize();
    for (auto g = c->graph_cache.begin(); g != c->graph_cache.end();) {
        if (g->first.graph_id == id) { (void)hipGraphExecDestroy(g->second); g = c->graph_cache.erase(g); }
        else ++g;
    }
    drop_call_graphs(c);
    free_graph(c, *it->second);
    c->graphs.erase(it);
    return SC_OK;
}

int sc_load_template(sc_ctx *c, int32_t t, const int32_t *edges, int32_t root, int32_t *tmpl_id) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
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
    std::lock_guard<std::recursive_mutex> lk(c->mu);
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
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (k < 1 || k > SC_MAX_K) return fail(c, SC_EINVAL, "k must be in [1, %d]", SC_MAX_K);
    c->k = k;
    c->seed = seed;
    return SC_OK;
}

int sc_set_option(sc_ctx *c, int32_t opt, int64_t v) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (serving(c) && opt != SC_OPT_GRAPH)
        return fail(c, SC_ESTATE, "options cannot change while the serving loop runs");
    switch (opt) {
    case SC_OPT_MAX_BATCH:
        if (v < 1 || v > SC_MAX_BATCH) return fail(c, SC_EINVAL, "max batch must be in [1, %d]", SC_MAX_BATCH);
        c->max_batch = v; return SC_OK;
    case SC_OPT_GRAPH:
        if (v < 0 || v > 2) return fail(c, SC_EINVAL, "graph option must be 0, 1 or 2");
        c->use_graph = v; return SC_OK;
    case SC_OPT_SEGMENT:
        if (v < 0 || v > (1 << 24)) return fail(c, SC_EINVAL, "segment must be in [0, 2^24]");
        if (v > 0 && v <= 64) return fail(c, SC_EINVAL, "segment must exceed 64");
        c->segment = v; return SC_OK;
    case SC_OPT_INTERLEAVE:
        if (v < 0 || v > 64 || (v & (v - 1))) return fail(c, SC_EINVAL, "interleave must be 0 or a power of two up to 64");
        c->interleave = v; return SC_OK;
    case SC_OPT_LDS_MAX:
        if (v != 0 && (v < 16384 || v > 163840)) return fail(c, SC_EINVAL, "LDS limit must be 0 or in [16384, 163840]");
        c->lds_max = v; return SC_OK;
    case SC_OPT_WAVE_ROW_MAX:
        if (v < -1 || v > 40960) return fail(c, SC_EINVAL, "wave row limit must be -1 (default) or in [0, 40960]");
        c->wave_row_max = v; return SC_OK;
    case SC_OPT_REORDER:
        if (v < 0 || v > 2) return fail(c, SC_EINVAL, "SC_OPT_REORDER must be 0, 1 or 2");
        c->reorder = v;
        return SC_OK;
    case SC_OPT_CHAIN:
        if (v < 0 || v > 1) return fail(c, SC_EINVAL, "SC_OPT_CHAIN must be 0 or 1");
        c->chain = v; return SC_OK;
    default: return fail(c, SC_EINVAL, "unknown option %d", opt);
    }
}

int sc_get_option(sc_ctx *c, int32_t opt, int64_t *v) {
    if (!c || !v) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    switch (opt) {
    case SC_OPT_MAX_BATCH: *v = c->max_batch; return SC_OK;
    case SC_OPT_GRAPH: *v = c->use_graph; return SC_OK;
    case SC_OPT_SEGMENT: *v = default_segment(c); return SC_OK;
    case SC_OPT_INTERLEAVE: *v = c->interleave; return SC_OK;
    case SC_OPT_LDS_MAX: *v = c->lds_max > 0 ? c->lds_max : ExecOpts().lds_max; return SC_OK;
    case SC_OPT_WAVE_ROW_MAX: *v = c->wave_row_max >= 0 ? c->wave_row_max : ExecOpts().wave_row_max; return SC_OK;
    case SC_OPT_REORDER: *v = c->reorder; return SC_OK;
    case SC_OPT_CHAIN: *v = c->chain; return SC_OK;
    default: return fail(c, SC_EINVAL, "unknown option %d", opt);
    }
}

int sc_plan_template(int32_t t, const int32_t *edges, int32_t root, int32_t k, int64_t n,
                     int64_t nnz, int32_t batch, sc_plan_info_t *out) {
    if (!out || batch < 1 || batch > SC_MAX_BATCH || n < 1 || nnz < 0) return SC_EINVAL;
    Plan P;
    std::string err;
    if (!choose_plan(t, edges, root, k, n, nnz, batch, ExecOpts(), P, err)) return SC_EINVAL;
    std::vector<int32_t> e;
    if (edges) e.assign(edges, edges + 2 * (t - 1));
    fill_plan_info(P, aut_of(t, e), out);
    return SC_OK;
}

int sc_plan_info(sc_ctx *c, int32_t gid, int32_t tid, int32_t n_colorings, sc_plan_info_t *out) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return fail(c, SC_EINVAL, "NULL argument");
    Plan P;
    int rc = pick_batch(c, gid, tid, c->k, std::max(1, n_colorings), 0, P);
    if (rc) return rc;
    fill_plan_info(P, c->tmpls[tid]->aut, out);
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

int sc_profile(sc_ctx *c, int32_t enable) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
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
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!n_out || (cap > 0 && !out)) return fail(c, SC_EINVAL, "NULL argument");
    std::vector<sc_kernel_stat_t> agg;
    for (auto &r : c->recs) {
        HIPCHK(c, hipEventSynchronize(r.b_ev));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.a_ev, r.b_ev));
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
        hit->layout_bytes += r.layout_bytes;
        hit->updates += r.updates;
    }
    *n_out = (int32_t)agg.size();
    for (int32_t i = 0; i < cap && i < (int32_t)agg.size(); ++i) out[i] = agg[i];
    return SC_OK;
}

int sc_valu_probe(sc_ctx *c, int32_t form, void *stream, double *mul_adds_per_s) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!mul_adds_per_s || form < 0 || form > 2) return fail(c, SC_EINVAL, "bad form or NULL output");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    DevMem out;
    int rc = dev_alloc(c, out, (size_t)kern::valu_probe_threads() * sizeof(uint64_t), st);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double madds = 0;
    float ms = 0.f;
    auto run = [&]() -> int {
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        auto *o = (unsigned long long *)out.p;
        HIPCHK(c, kern::launch_valu_probe(form, 1, 256, o, &madds, st));          // warm
        HIPCHK(c, hipEventRecord(e0, st));
        HIPCHK(c, kern::launch_valu_probe(form, 2, 16384, o, &madds, st));
        HIPCHK(c, hipEventRecord(e1, st));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        return SC_OK;
    };
    rc = run();
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(c, out);
    if (rc) return rc;
    if (ms <= 0.f) return fail(c, SC_EDEVICE, "probe time not measured");
    *mul_adds_per_s = madds / (ms * 1e-3);
    return SC_OK;
}

int sc_profile_launches(sc_ctx *c, sc_launch_t *out, int32_t cap, int32_t *n_out) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!n_out || (cap > 0 && !out)) return fail(c, SC_EINVAL, "NULL argument");
    *n_out = (int32_t)c->recs.size();
    for (int32_t i = 0; i < cap && i < (int32_t)c->recs.size(); ++i) {
        const auto &r = c->recs[i];
        HIPCHK(c, hipEventSynchronize(r.b_ev));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.a_ev, r.b_ev));
        sc_launch_t &o = out[i];
        std::memset(&o, 0, sizeof o);
        std::snprintf(o.kernel, sizeof o.kernel, "%s", r.kernel.c_str());
        std::snprintf(o.family, sizeof o.family, "%s", r.name);
        o.step = r.step; o.h = r.h; o.a = r.a; o.p = r.p; o.colorings = r.colorings;
        o.ms = ms;
        o.alg_bytes = r.bytes;
        o.layout_bytes = r.layout_bytes;
        o.updates = r.updates;
    }
    return SC_OK;
}

}  // extern "C"
