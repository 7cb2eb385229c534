// libsc executor: one pass = colourings first..first+B-1 folded into the table
// columns, run as the plan's kernel sequence (directly, or replayed from a
// captured hipGraph).  sc_run chains passes without host round trips;
// sc_run_batch does the same for many (graph, template, k, seed) jobs at
// once; sc_autotune picks the interleave and LDS limit by timing real passes.
#include <algorithm>
#include <climits>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>

#include "rt.h"

namespace sc {

namespace {

std::atomic<uint64_t> g_buffer_generation{1};

hipEvent_t next_event(sc_ctx *c) {
    if (c->events_used == c->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->event_pool.push_back(e);
    }
    return c->event_pool[c->events_used++];
}

// What a traced launch belongs to: its family, the DP step (index and sizes;
// step -1 for launches outside the steps), the colourings of the pass, the
// compulsory bytes of the paper's layout and of the rooted-colour layout, and
// its updates in the paper's units.
struct LaunchInfo {
    const char *family;
    int step = -1, h = 0, a = 0, p = 0, colorings = 0;
    double bytes = 0, layout_bytes = 0, updates = 0;
};

// Brackets one launch with HIP events on its stream while profiling is on and
// records the kernel instantiation the launcher enqueued.
struct ProfScope {
    sc_ctx *c;
    hipStream_t st;
    LaunchInfo li;
    hipEvent_t a = nullptr;
    ProfScope(sc_ctx *c_, bool on, hipStream_t st_, const LaunchInfo &l) : c(c_), st(st_), li(l) {
        if (on && (a = next_event(c))) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = next_event(c);
        if (!b) return;
        (void)hipEventRecord(b, st);
        c->recs.push_back({li.family, kern::last_kernel_name(), li.step, li.h, li.a, li.p, li.colorings, a, b,
                           li.bytes, li.layout_bytes, li.updates});
    }
};

int ensure_gen(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st, PassBuffers &b) {
    if (m.p && m.bytes >= bytes) return SC_OK;
    uint64_t dummy = 0;
    int rc = ensure(c, m, bytes, st, &dummy);
    b.gen = g_buffer_generation.fetch_add(1);
    return rc;
}

// Kernel shape and device index tables of one step: the tables are the staged
// copies when `staged` is given, else the context's (uploaded on first use, so
// prepare_pass calls this before any capture).
int step_args(sc_ctx *c, const Plan &P, const Step &s, uint64_t mod, kern::StepShape &sh,
              kern::StepTables &tb, const StagedTables *staged = nullptr) {
    const int k = P.k;
    sh.k = k; sh.a = s.a; sh.p = s.p;
    sh.B = P.batch; sh.Bi = P.interleave;
    sh.Wq = s.p >= 2 ? (int)binom(k - 1, s.p - 1) : 0;
    sh.Wn = (int)binom(k - 1, s.p);
    sh.Wa = (int)binom(k - 1, s.a - 1);
    sh.Wh = (int)binom(k - 1, s.h - 1);
    sh.nsplit = (int)binom(s.h - 1, s.a - 1);
    sh.amode = s.amode;
    sh.wave_row_max = P.opts.wave_row_max;
    sh.mod = mod;
    if (staged) {
        auto find = [](const auto &m, const TableKey &key, auto *&out) {
            auto it = m.find(key);
            if (it == m.end()) return false;
            out = it->second;
            return true;
        };
        if (s.a > 1 && !find(staged->split, TableKey{k - 1, s.h - 1, s.a - 1}, tb.split))
            return fail(c, SC_EINVAL, "split table (%d,%d,%d) not staged", k - 1, s.h - 1, s.a - 1);
        if (s.p > 1) {
            if (!find(staged->unrank, TableKey{k - 1, s.p - 1, 0}, tb.unrank) ||
                !find(staged->rank, TableKey{k - 1, 0, 0}, tb.rank))
                return fail(c, SC_EINVAL, "rank tables for k-1=%d, size %d not staged", k - 1, s.p - 1);
            tb.n_rank = kern::rank_entries(k - 1);
        }
        return SC_OK;
    }
    int rc;
    if (s.a > 1 && (rc = get_split(c, k - 1, s.h - 1, s.a - 1, &tb.split))) return rc;
    if (s.p > 1) {
        if ((rc = get_unrank(c, k - 1, s.p - 1, &tb.unrank))) return rc;
        if ((rc = get_rank(c, k - 1, &tb.rank))) return rc;
        tb.n_rank = kern::rank_entries(k - 1);
    }
    return SC_OK;
}

// Shape and split tables of one chain (tables uploaded on first use, or the
// staged copies).
int chain_args(sc_ctx *c, const Plan &P, const Chain &ch, uint64_t mod, kern::ChainShape &cs,
               const StagedTables *staged) {
    const int k = P.k;
    const Step &s0 = P.steps[ch.first];
    cs.k = k; cs.a0 = s0.a; cs.steps = ch.last - ch.first + 1;
    cs.B = P.batch; cs.Bi = P.interleave; cs.wmax = ch.wmax; cs.mod = mod;
    for (int i = 0; i < cs.steps; ++i) {
        const Step &s = P.steps[ch.first + i];
        kern::StepShape sh;
        kern::StepTables tb;
        if (int rc = step_args(c, P, s, mod, sh, tb, staged)) return rc;
        cs.Wa[i] = sh.Wa; cs.Wh[i] = sh.Wh; cs.nsplit[i] = sh.nsplit; cs.split[i] = tb.split;
    }
    return SC_OK;
}

}  // namespace

size_t npre_bytes(const Graph &g, const Plan &P) {
    size_t w = 0;
    for (const Step &s : P.steps) w = std::max(w, (size_t)g.n_split * binom(P.k - 1, s.p) * P.batch);
    return w * 8;
}

uint64_t buffers_after(const Graph &g, const Plan &P, const PassBuffers &b) {
    auto grown = [](const DevMem &m, uint64_t need) { return std::max<uint64_t>(m.bytes, need); };
    return grown(b.arena, P.arena_bytes) + grown(b.colbuf, (uint64_t)g.n_rows * P.batch) +
           grown(b.npre, npre_bytes(g, P)) + grown(b.xbuf, (SC_MAX_BATCH + 1) * sizeof(uint64_t)) +
           grown(b.desc, 2 * sizeof(uint64_t));
}

int prepare_pass(sc_ctx *c, const PassSpec &s, PassBuffers &b, hipStream_t st) {
    Graph &g = *s.g;
    const Plan &P = *s.P;
    int rc;
    if ((rc = rebin(c, g, plan_segment(c, P)))) return rc;
    if ((rc = ensure_gen(c, b.arena, P.arena_bytes, st, b))) return rc;
    if ((rc = ensure_gen(c, b.colbuf, (size_t)g.n_rows * P.batch, st, b))) return rc;
    if ((rc = ensure_gen(c, b.xbuf, (SC_MAX_BATCH + 1) * sizeof(uint64_t), st, b))) return rc;
    if ((rc = ensure_gen(c, b.desc, 2 * sizeof(uint64_t), st, b))) return rc;
    const size_t np = npre_bytes(g, P);
    if (np && (rc = ensure_gen(c, b.npre, np, st, b))) return rc;
    for (int si = 0; si < (int)P.steps.size(); ++si) {
        kern::StepShape sh;
        kern::StepTables tb;
        if ((rc = step_args(c, P, P.steps[si], s.mod, sh, tb))) return rc;
    }
    return SC_OK;
}

// One chain of single-vertex attaches (steps ch.first..ch.last): the split
// pre-pass of its first step (the colour counts of rows above the segment
// size), then the chain kernel.
template <typename BufOf>
int enqueue_chain(sc_ctx *c, const PassSpec &sp, const Chain &ch, const kern::GraphBins &bins,
                  const uint8_t *col, const BufOf &buf, uint64_t *Npre, unsigned long long *flags,
                  const StagedTables *staged, hipStream_t st, bool prof) {
    const Plan &P = *sp.P;
    const Graph &g = *sp.g;
    const int B = P.batch, k = P.k;
    const double dn = (double)g.n_rows, dB = (double)B, nall = (double)g.n, nnz = (double)g.nnz;
    const Step &s0 = P.steps[ch.first], &sl = P.steps[ch.last];
    int rc;
    kern::StepShape sh;
    kern::StepTables tb;
    if ((rc = step_args(c, P, s0, sp.mod, sh, tb, staged))) return rc;
    kern::ChainShape cs;
    if ((rc = chain_args(c, P, ch, sp.mod, cs, staged))) return rc;
    LaunchInfo li{"chain", ch.first, sl.h, s0.a, 1, B};
    for (int i = 0; i < cs.steps; ++i) {
        const Step &s = P.steps[ch.first + i];
        li.updates += (nnz * (double)k + nall * (double)binom(k, s.h) * (s.a > 1 ? (double)binom(s.h, s.a) : 1.0)) * dB;
    }
    // compulsory bytes of the fused chain: the adjacency and colours once, the
    // first step's active table read once, the last step's output written
    // once (the intermediate tables never leave the kernel)
    li.bytes = 4.0 * nnz + 8.0 * (nall + 1) + nall * dB + (s0.a > 1 ? 8.0 * nall * dB * (double)binom(k, s0.a) : 0.0) +
               8.0 * nall * dB * (double)binom(k, sl.h);
    li.layout_bytes = 4.0 * nnz + 8.0 * (dn + 1) + dn * dB + 8.0 * dn * dB * ((s0.a > 1 ? cs.Wa[0] : 0) + cs.Wh[cs.steps - 1]) +
                      8.0 * (double)g.n_split * sh.Wn * dB;
    if (g.n_split) {
        LaunchInfo ls{"split", ch.first, s0.h, s0.a, 1, B};
        ls.layout_bytes = 4.0 * g.split_nnz + 16.0 * g.n_split * sh.Wn * dB;
        ProfScope ps(c, prof, st, ls);
        HIPCHK(c, kern::launch_dp_split(bins, sh, tb, col, nullptr, Npre, flags, st));
    }
    ProfScope ps(c, prof, st, li);
    HIPCHK(c, kern::launch_dp_chain(bins, cs, col, buf(s0.buf_a), Npre, buf(sl.buf_s), flags,
                                    P.opts.wave_row_max, st));
    return SC_OK;
}

int enqueue_pass(sc_ctx *c, const PassSpec &sp, PassBuffers &pb, hipStream_t st, bool prof) {
    Graph &g = *sp.g;
    const Plan &P = *sp.P;
    const int B = P.batch, k = P.k;
    const int64_t n = g.n_rows;
    const double dn = (double)n, dB = (double)B;
    int rc;
    auto *X = (unsigned long long *)pb.xbuf.p;
    auto *flags = X + SC_MAX_BATCH;
    auto *col = (uint8_t *)pb.colbuf.p;
    auto *base = (uint8_t *)pb.arena.p;
    auto *Npre = (uint64_t *)pb.npre.p;
    auto buf = [&](int id) { return id < 0 ? (uint64_t *)nullptr : (uint64_t *)(base + P.bufs[id].offset); };
    const kern::GraphBins bins = bins_of(g);
    // the paper's units count every vertex of the graph (isolated ones included)
    const double nall = (double)g.n, nnz = (double)g.nnz;

    {
        LaunchInfo li{"zero"};
        li.colorings = B;
        ProfScope ps(c, prof, st, li);
        HIPCHK(c, kern::launch_zero_u64((uint64_t *)X, SC_MAX_BATCH + 1, st));
    }
    {
        LaunchInfo li{"color"};
        li.colorings = B;
        li.bytes = li.layout_bytes = dn * B;
        ProfScope ps(c, prof, st, li);
        HIPCHK(c, kern::launch_color((const uint64_t *)pb.desc.p, n, B, k, (const int32_t *)g.perm.p, col, st));
    }
    const Step *last = nullptr;
    size_t next_chain = 0;
    for (int si = 0; si < (int)P.steps.size(); ++si) {
        const Step &s = P.steps[si];
        if (next_chain < P.chains.size() && P.chains[next_chain].first == si) {
            const Chain &ch = P.chains[next_chain++];
            if ((rc = enqueue_chain(c, sp, ch, bins, col, buf, Npre, flags, pb.staged, st, prof))) return rc;
            last = &P.steps[ch.last];
            si = ch.last;
            continue;
        }
        kern::StepShape sh;
        kern::StepTables tb;
        if ((rc = step_args(c, P, s, sp.mod, sh, tb, pb.staged))) return rc;
        uint64_t *S = buf(s.buf_s);
        const uint64_t *Pp = buf(s.buf_p), *A = buf(s.buf_a);
        LaunchInfo li{s.p == 1 ? "row_hist" : "row_gather", si, s.h, s.a, s.p, B};
        // updates in the paper's units (Lemma 1): nnz*C(k,p) neighbour-sum
        // updates, n*C(k,h)*C(h,a) multiply-adds (n*C(k,h) selects for a = 1)
        const double Wp = (double)binom(k, s.p), Wa = (double)binom(k, s.a), Wh = (double)binom(k, s.h);
        li.updates = (nnz * Wp + nall * Wh * (s.a > 1 ? (double)binom(s.h, s.a) : 1.0)) * dB;
        // compulsory bytes of the fused step in the paper's layout (every
        // vertex, binom(k, s) colour sets per row): the adjacency once, the
        // passive table read once (colours for p = 1), the active table read
        // once (colours for a = 1), the output written once; N never stored
        li.bytes = 4.0 * nnz + 8.0 * (nall + 1) + (s.p > 1 ? 8.0 * nall * dB * Wp : nall * dB) +
                   (s.a > 1 ? 8.0 * nall * dB * Wa : nall * dB) + 8.0 * nall * dB * Wh;
        // the same in the rooted-colour layout over the table rows, plus the
        // split rows' sums written and read back
        const bool pre = g.n_split && !kern::root_step(sh);      // the root step sums every row itself
        li.layout_bytes = 4.0 * nnz + 8.0 * (dn + 1) + dn * dB +
                          8.0 * dn * dB * ((s.p > 1 ? sh.Wq : 0) + (s.a > 1 ? sh.Wa : 0) + sh.Wh) +
                          (pre ? 8.0 * (double)g.n_split * sh.Wn * dB : 0.0);
        if (pre) {
            // the heavy rows' share of the step's neighbour sums; its bytes
            // and updates are counted with the row kernel, which completes them
            LaunchInfo ls{"split", si, s.h, s.a, s.p, B};
            ls.layout_bytes = 4.0 * g.split_nnz + 16.0 * g.n_split * sh.Wn * dB;
            ProfScope ps(c, prof, st, ls);
            HIPCHK(c, kern::launch_dp_split(bins, sh, tb, col, Pp, Npre, flags, st));
        }
        {
            ProfScope ps(c, prof, st, li);
            HIPCHK(c, kern::launch_dp_row(bins, sh, tb, col, Pp, A, Npre, S, flags, st));
        }
        last = &s;
    }
    const int W = (int)binom(k - 1, last->h - 1);
    LaunchInfo li{"reduce"};
    li.colorings = B;
    li.layout_bytes = 8.0 * dn * W * B;
    li.bytes = 8.0 * nall * (double)binom(k, last->h) * B;
    ProfScope ps(c, prof, st, li);
    HIPCHK(c, kern::launch_reduce(n, buf(last->buf_s), W, B, P.interleave, sp.mod, X, flags, st));
    return SC_OK;
}

void unpack_pass(const uint64_t *host_res, int B, uint64_t *counts, uint8_t *flags) {
    for (int r = 0; r < B; ++r) {
        counts[r] = host_res[r];
        flags[r] = (uint8_t)((host_res[SC_MAX_BATCH] >> r) & 1);
    }
}

int launch_pass(sc_ctx *c, int gid, int tid, const PassSpec &s, PassBuffers &b, hipStream_t st,
                uint64_t *host_desc, uint64_t *host_res, bool allow_graph) {
    const Plan &P = *s.P;
    if (P.steps.empty() || s.g->n_rows == 0) {   // t = 1: every vertex is a map; no edge: no map
        for (int r = 0; r < SC_MAX_BATCH; ++r) host_res[r] = P.steps.empty() ? (uint64_t)s.g->n : 0;
        host_res[SC_MAX_BATCH] = 0;
        return SC_OK;
    }
    int rc;
    if ((rc = prepare_pass(c, s, b, st))) return rc;
    host_desc[0] = s.seed;
    host_desc[1] = s.first;
    HIPCHK(c, hipMemcpyAsync(b.desc.p, host_desc, 2 * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if (allow_graph && c->use_graph && !c->prof) {
        GraphExecKey key{gid, tid, P.k, P.batch, P.interleave, P.opts.lds_max, P.opts.wave_row_max,
                         s.g->seg, P.opts.chain, s.mod, b.gen};
        auto it = c->graph_cache.find(key);
        if (it == c->graph_cache.end()) {
            hipGraph_t graph = nullptr;
            HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
            rc = enqueue_pass(c, s, b, st, false);
            hipError_t e = hipStreamEndCapture(st, &graph);
            if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
            if (e != hipSuccess) return fail(c, SC_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(c, SC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
            it = c->graph_cache.emplace(key, exec).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second, st));
    } else {
        if ((rc = enqueue_pass(c, s, b, st, c->prof))) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(host_res, b.xbuf.p, (SC_MAX_BATCH + 1) * sizeof(uint64_t),
                             hipMemcpyDeviceToHost, st));
    return SC_OK;
}

}  // namespace sc

using namespace sc;

namespace sc {

constexpr size_t kStageWords = 2 + SC_MAX_BATCH + 1;   // descriptor + results of one pass
constexpr size_t kResWords = SC_MAX_BATCH + 1;         // results of one pass
constexpr size_t kMaxCallGraphs = 64;                  // whole-call graphs kept at once

void drop_call_graphs(sc_ctx *c) {
    for (auto &kv : c->call_graphs) (void)hipGraphExecDestroy(kv.second);
    c->call_graphs.clear();
}

namespace {

// SC_OPT_GRAPH = 2: every pass of the call in one captured graph, replayed
// with one launch.  The passes run back to back on the shared buffers (sized
// for the largest pass beforehand); pass i reads its seed and first colouring
// from call_desc[2i..] and leaves its sums and flags in call_x[i][..].  Every
// pass is prepared first (bins, index tables), so nothing allocates while the
// stream is captured.
int run_passes_one_graph(sc_ctx *c, std::vector<PassJob> &passes, hipStream_t st,
                         const std::function<void(const PassJob &, const uint64_t *)> &done) {
    int rc;
    PassBuffers &b = c->main;
    const size_t np = passes.size();
    std::vector<PassSpec> specs(np);
    std::vector<GraphExecKey> key(np);
    for (size_t i = 0; i < np; ++i) {
        PassJob &p = passes[i];
        PassSpec &s = specs[i];
        s.g = c->graphs[p.gid].get();
        s.P = &p.P;
        s.k = p.k; s.seed = p.seed; s.first = p.first; s.mod = p.mod;
        if ((rc = prepare_pass(c, s, b, st))) return rc;
    }
    if (c->call_desc.bytes < np * 2 * sizeof(uint64_t) || c->call_x.bytes < np * kResWords * sizeof(uint64_t))
        ++c->call_gen;
    if ((rc = ensure(c, c->call_desc, np * 2 * sizeof(uint64_t), st))) return rc;
    if ((rc = ensure(c, c->call_x, np * kResWords * sizeof(uint64_t), st))) return rc;
    for (size_t i = 0; i < np; ++i) {
        const Plan &P = passes[i].P;
        key[i] = GraphExecKey{passes[i].gid, passes[i].tid, P.k, P.batch, P.interleave, P.opts.lds_max,
                              P.opts.wave_row_max, plan_segment(c, P), P.opts.chain, passes[i].mod, b.gen};
    }
    auto ck = std::make_pair(key, c->call_gen);
    auto it = c->call_graphs.find(ck);
    if (it == c->call_graphs.end()) {
        if (c->call_graphs.size() >= kMaxCallGraphs) {
            HIPCHK(c, hipStreamSynchronize(st));
            drop_call_graphs(c);
        }
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        for (size_t i = 0; i < np && !rc; ++i) {
            // the pass's bins exist (prepare_pass built them): this only swaps them in
            if ((rc = rebin(c, *specs[i].g, plan_segment(c, passes[i].P), false))) break;
            PassBuffers v = b;
            v.desc.p = (uint64_t *)c->call_desc.p + 2 * i;
            v.xbuf.p = (uint64_t *)c->call_x.p + kResWords * i;
            rc = enqueue_pass(c, specs[i], v, st, false);
        }
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(c, SC_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(c, SC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        it = c->call_graphs.emplace(ck, exec).first;
    }
    uint64_t *desc = c->host_out, *res = c->host_out + 2 * np;
    for (size_t i = 0; i < np; ++i) {
        desc[2 * i] = passes[i].seed;
        desc[2 * i + 1] = passes[i].first;
    }
    HIPCHK(c, hipMemcpyAsync(c->call_desc.p, desc, np * 2 * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipGraphLaunch(it->second, st));
    HIPCHK(c, hipMemcpyAsync(res, c->call_x.p, np * kResWords * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (size_t i = 0; i < np; ++i) done(passes[i], res + kResWords * i);
    return SC_OK;
}

}  // namespace

// Plans every pass of the jobs, runs them back to back on `st` and waits once.
int run_passes(sc_ctx *c, std::vector<PassJob> &passes, hipStream_t st,
               const std::function<void(const PassJob &, const uint64_t *)> &done) {
    int rc;
    if ((rc = host_staging(c, std::max<size_t>(1, passes.size()) * kStageWords))) return rc;
    // size the buffers for the largest pass first, so no buffer moves mid-chain
    size_t arena = 0, colb = 0, npre = 0;
    bool trivial = false;
    for (auto &p : passes) {
        const Graph &g = *c->graphs[p.gid];
        arena = std::max<size_t>(arena, p.P.arena_bytes);
        colb = std::max<size_t>(colb, (size_t)g.n_rows * p.P.batch);
        npre = std::max<size_t>(npre, npre_bytes(g, p.P));
        trivial |= p.P.steps.empty() || g.n_rows == 0;
    }
    PassBuffers &b = c->main;
    if ((rc = ensure_gen(c, b.arena, arena, st, b))) return rc;
    if ((rc = ensure_gen(c, b.colbuf, colb, st, b))) return rc;
    if (npre && (rc = ensure_gen(c, b.npre, npre, st, b))) return rc;
    if (c->use_graph == 2 && !c->prof && !trivial && !passes.empty())
        return run_passes_one_graph(c, passes, st, done);
    for (size_t i = 0; i < passes.size(); ++i) {
        auto &p = passes[i];
        PassSpec s;
        s.g = c->graphs[p.gid].get();
        s.P = &p.P;
        s.k = p.k;
        s.seed = p.seed;
        s.first = p.first;
        s.mod = p.mod;
        uint64_t *stage = c->host_out + i * kStageWords;
        if ((rc = launch_pass(c, p.gid, p.tid, s, b, st, stage, stage + 2, true))) return rc;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    for (size_t i = 0; i < passes.size(); ++i) done(passes[i], c->host_out + i * kStageWords + 2);
    return SC_OK;
}

bool single_chain(const Plan &P) {
    return P.steps.size() >= 2 && P.chains.size() == 1 && P.chains[0].first == 0 &&
           P.chains[0].last == (int)P.steps.size() - 1 && P.steps[0].a == 1;
}

int run_wide_passes(sc_ctx *c, std::vector<PassJob> &passes, const std::vector<int> &limbs, hipStream_t st,
                    const std::function<void(const PassJob &, const uint64_t *, uint64_t)> &done) {
    int rc;
    if (limbs.empty()) return fail(c, SC_EINVAL, "no limbs for the exact multi-limb pass");
    const int L = limbs.back();
    const size_t words = (size_t)SC_MAX_BATCH * (L + 1) + 1;          // sums, then the flag word
    if ((rc = host_staging(c, std::max<size_t>(1, passes.size()) * (words + 2)))) return rc;
    PassBuffers &b = c->main;
    for (size_t i = 0; i < passes.size(); ++i) {
        PassJob &pj = passes[i];
        Graph &g = *c->graphs[pj.gid];
        if (pj.P.steps.size() != limbs.size())
            return fail(c, SC_EINVAL, "limbs given for %zu steps, the plan has %zu", limbs.size(), pj.P.steps.size());
        // the interleave whose two widest intermediate rows fit the LDS limit
        const int k1 = pj.k - 1;
        int wrow = 0;
        for (size_t j = 1; j + 1 < limbs.size(); ++j)
            wrow = std::max(wrow, (int)binom(k1, pj.P.steps[j].h - 1) * limbs[j]);
        int bi = pj.P.interleave;
        while (bi > 1 && kern::chain_wide_lds_bytes(k1, wrow, bi) > pj.P.opts.lds_max) bi /= 2;
        if (bi != pj.P.interleave) {
            ExecOpts o = pj.P.opts;
            o.interleave = bi;
            Plan P2;
            if ((rc = make_plan(c, g, *c->tmpls[pj.tid], o, pj.k, pj.P.batch, P2))) return rc;
            pj.P = std::move(P2);
        }
        const Plan &P = pj.P;
        if (!single_chain(P)) return fail(c, SC_EINVAL, "the exact multi-limb pass needs a single-chain plan");
        PassSpec sp;
        sp.g = &g; sp.P = &P; sp.k = pj.k; sp.seed = pj.seed; sp.first = pj.first;
        if ((rc = prepare_pass(c, sp, b, st))) return rc;
        const uint64_t W = binom(pj.k - 1, P.steps.back().h - 1);
        if ((rc = ensure(c, c->wide_tab, (size_t)g.n_rows * W * P.batch * L * 8, st))) return rc;
        if ((rc = ensure(c, c->wide_x, words * 8, st))) return rc;
        auto *X = (unsigned long long *)c->wide_x.p;
        auto *flags = X + (size_t)SC_MAX_BATCH * (L + 1);
        uint64_t *stage = c->host_out + i * (words + 2);
        stage[0] = pj.seed;
        stage[1] = pj.first;
        HIPCHK(c, hipMemcpyAsync(b.desc.p, stage, 2 * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        HIPCHK(c, kern::launch_zero_u64((uint64_t *)X, (int64_t)words, st));
        auto *col = (uint8_t *)b.colbuf.p;
        HIPCHK(c, kern::launch_color((const uint64_t *)b.desc.p, g.n_rows, P.batch, pj.k, (const int32_t *)g.perm.p,
                                     col, st));
        const kern::GraphBins bins = bins_of(g);
        kern::ChainShape cs;
        if ((rc = chain_args(c, P, P.chains[0], 0, cs, nullptr))) return rc;
        kern::StepShape sh;
        kern::StepTables tb;
        if ((rc = step_args(c, P, P.steps[0], 0, sh, tb))) return rc;
        if (g.n_split) HIPCHK(c, kern::launch_dp_split(bins, sh, tb, col, nullptr, (uint64_t *)b.npre.p, flags, st));
        auto *S = (uint64_t *)c->wide_tab.p;
        HIPCHK(c, kern::launch_dp_chain_wide(bins, cs, limbs.data(), col, (const uint64_t *)b.npre.p, S, flags,
                                             P.opts.wave_row_max, st));
        HIPCHK(c, kern::launch_reduce_wide(g.n_rows, S, (int)W, P.batch, P.interleave, L, X, st));
        HIPCHK(c, hipMemcpyAsync(stage + 2, X, words * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(c, hipStreamSynchronize(st));
    for (size_t i = 0; i < passes.size(); ++i) {
        const uint64_t *stage = c->host_out + i * (words + 2) + 2;
        done(passes[i], stage, stage[(size_t)SC_MAX_BATCH * (L + 1)]);
    }
    return SC_OK;
}

int check_coloring_range(sc_ctx *c, uint64_t first, int64_t n) {
    if (n < 0 || first > SC_MAX_COLORING || (uint64_t)n > SC_MAX_COLORING - first)
        return fail(c, SC_EINVAL, "colourings %llu..%llu+%lld reach past 2^24, where the colouring rule repeats",
                    (unsigned long long)first, (unsigned long long)first, (long long)n);
    return SC_OK;
}

// Splits n colourings of one job into passes of the planned batch.
int plan_job(sc_ctx *c, int job, int gid, int tid, int k, uint64_t seed, uint64_t first, int n,
             std::vector<PassJob> &out) {
    if (int rc = check_coloring_range(c, first, n)) return rc;
    int off = 0;
    while (off < n) {
        PassJob p;
        p.job = job; p.gid = gid; p.tid = tid; p.k = k; p.seed = seed;
        p.first = first + (uint64_t)off;
        p.offset = off;
        int rc = pick_batch(c, gid, tid, k, n - off, 0, p.P);
        if (rc) return rc;
        off += p.P.batch;
        out.push_back(std::move(p));
    }
    return SC_OK;
}

int check_run_args(sc_ctx *c, int gid, int tid, int ncol) {
    if (ncol < 0) return fail(c, SC_EINVAL, "n_colorings < 0");
    auto gi = c->graphs.find(gid);
    if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", gid);
    auto ti = c->tmpls.find(tid);
    if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", tid);
    if (c->k < ti->second->t) return fail(c, SC_EINVAL, "k=%d < t=%d (call sc_set_colors)", c->k, ti->second->t);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    return SC_OK;
}

}  // namespace sc

namespace sc {

void estimates(const uint64_t *counts, const uint8_t *ovf, int n, int k, int t, double aut,
               double *maps, double *copies) {
    bool any = false;
    double sum = 0;
    for (int i = 0; i < n; ++i) { any |= ovf[i] != 0; sum += (double)counts[i]; }
    double m = NAN, cp = NAN;
    if (n > 0 && !any) {
        m = sum / n / colorful_probability(k, t);
        cp = m / aut;
    }
    if (maps) *maps = m;
    if (copies) *copies = cp;
}

}  // namespace sc

extern "C" {

int sc_run(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, int32_t ncol, void *stream,
           uint64_t *counts, uint8_t *overflow, double *est_maps, double *est_copies) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (ncol < 0) return fail(c, SC_EINVAL, "n_colorings < 0");
    if (ncol > 0 && (!counts || !overflow)) return fail(c, SC_EINVAL, "NULL output");
    auto gi = c->graphs.find(gid);
    if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", gid);
    auto ti = c->tmpls.find(tid);
    if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", tid);
    if (c->k < ti->second->t) return fail(c, SC_EINVAL, "k=%d < t=%d (call sc_set_colors)", c->k, ti->second->t);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    std::vector<PassJob> passes;
    int rc = plan_job(c, 0, gid, tid, c->k, c->seed, first, ncol, passes);
    if (rc) return rc;
    rc = run_passes(c, passes, st, [&](const PassJob &p, const uint64_t *res) {
        unpack_pass(res, p.P.batch, counts + p.offset, overflow + p.offset);
    });
    if (rc) return rc;
    estimates(counts, overflow, ncol, c->k, ti->second->t, ti->second->aut, est_maps, est_copies);
    return SC_OK;
}

int sc_run_batch(sc_ctx *c, sc_job_t *jobs, int32_t n_jobs, void *stream) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(c, SC_EINVAL, "bad job array");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    std::vector<PassJob> passes;
    int first_err = SC_OK;
    std::string first_msg;
    for (int j = 0; j < n_jobs; ++j) {
        sc_job_t &J = jobs[j];
        J.status = SC_OK;
        J.est_maps = J.est_copies = NAN;
        int rc = SC_OK;
        if (J.n_colorings < 0 || (J.n_colorings > 0 && (!J.counts || !J.overflow)))
            rc = fail(c, SC_EINVAL, "job %d: bad colouring count or NULL output", j);
        std::vector<PassJob> mine;
        if (!rc) rc = plan_job(c, j, J.graph_id, J.tmpl_id, J.k, J.seed, J.first_coloring, J.n_colorings, mine);
        if (rc) {
            J.status = rc;
            if (!first_err) { first_err = rc; first_msg = c->err; }
            continue;
        }
        for (auto &p : mine) passes.push_back(std::move(p));
    }
    int rc = run_passes(c, passes, st, [&](const PassJob &p, const uint64_t *res) {
        sc_job_t &J = jobs[p.job];
        unpack_pass(res, p.P.batch, J.counts + p.offset, J.overflow + p.offset);
    });
    if (rc) {
        for (int j = 0; j < n_jobs; ++j) if (jobs[j].status == SC_OK) jobs[j].status = rc;
        return rc;
    }
    for (int j = 0; j < n_jobs; ++j) {
        sc_job_t &J = jobs[j];
        if (J.status) continue;
        const Template &T = *c->tmpls[J.tmpl_id];
        estimates(J.counts, J.overflow, J.n_colorings, J.k, T.t, T.aut, &J.est_maps, &J.est_copies);
    }
    if (first_err) c->err = first_msg;
    return first_err;
}

int sc_autotune(sc_ctx *c, int32_t gid, int32_t tid, int32_t n_colorings, sc_tune_t *out) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return fail(c, SC_EINVAL, "NULL argument");
    Plan P;
    int rc = pick_batch(c, gid, tid, c->k, std::max(1, n_colorings), 0, P);
    if (rc) return rc;
    const int B = P.batch;
    const TuneKey key{gid, tid, c->k, B};
    c->tuned.erase(key);
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    Tuned best;
    best.ms = 1e300;
    int trials = 0;
    // one pass of the planned batch with the candidate knobs, after a warm-up pass
    auto trial = [&](const Tuned &cand) -> int {
        c->tuned[key] = cand;
        std::vector<PassJob> passes;
        int r;
        if ((r = plan_job(c, 0, gid, tid, c->k, c->seed, 0, B, passes))) return r;
        auto sink = [&](const PassJob &, const uint64_t *) {};
        if ((r = run_passes(c, passes, c->stream, sink))) return r;
        HIPCHK(c, hipEventRecord(e0, c->stream));
        if ((r = run_passes(c, passes, c->stream, sink))) return r;
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        ++trials;
        if (ms < best.ms) { best = cand; best.ms = ms; }
        return SC_OK;
    };
    // 1. interleave caps (the four largest powers of two dividing the batch)
    //    and row-kernel LDS limits, at the default segment and row threshold
    std::vector<int> inter;
    for (int bi = 64; bi >= 1 && inter.size() < 4; bi /= 2)
        if (B % bi == 0) inter.push_back(bi);
    static const int ldss[] = {32 * 1024, 64 * 1024, 96 * 1024, 128 * 1024};
    for (int bi : inter)
        for (int lm : ldss) {
            if (rc) break;
            Tuned cand;
            cand.interleave = bi;
            cand.lds_max = lm;
            rc = trial(cand);
        }
    // 2. neighbours per split-row work item, then 3. the per-row LDS up to
    //    which a wavefront builds a row alone, each around the best so far
    static const int segs[] = {256, 1024, 2048};
    const Tuned base1 = best;
    for (int sg : segs) {
        if (rc) break;
        Tuned cand = base1;
        cand.seg = sg;
        rc = trial(cand);
    }
    static const int waves[] = {0, 16384};
    const Tuned base2 = best;
    for (int wr : waves) {
        if (rc) break;
        Tuned cand = base2;
        cand.wave_row_max = wr;
        rc = trial(cand);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) { c->tuned.erase(key); return rc; }
    c->tuned[key] = best;
    out->interleave = best.interleave;
    out->lds_max = best.lds_max;
    out->seg = best.seg > 0 ? best.seg : default_segment(c);
    out->wave_row_max = best.wave_row_max >= 0 ? best.wave_row_max : ExecOpts().wave_row_max;
    out->batch = B;
    out->ms = best.ms;
    out->trials = trials;
    return SC_OK;
}

int sc_tune_save(sc_ctx *c, const char *path) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!path) return fail(c, SC_EINVAL, "NULL path");
    FILE *f = fopen(path, "w");
    if (!f) return fail(c, SC_EINVAL, "cannot write %s", path);
    for (auto &kv : c->tuned) {
        auto gi = c->graphs.find(std::get<0>(kv.first));
        auto ti = c->tmpls.find(std::get<1>(kv.first));
        if (gi == c->graphs.end() || ti == c->tmpls.end()) continue;
        const Graph &g = *gi->second;
        const Template &T = *ti->second;
        fprintf(f, "%lld %lld %lld %d %d %d %d %d %d %d %.6f", (long long)g.n, (long long)g.nnz,
                (long long)g.max_deg, std::get<2>(kv.first), std::get<3>(kv.first),
                kv.second.interleave, kv.second.lds_max, kv.second.seg, kv.second.wave_row_max, T.t,
                kv.second.ms);
        for (int32_t e : T.edges) fprintf(f, " %d", e);
        fprintf(f, "\n");
    }
    fclose(f);
    return SC_OK;
}

int sc_tune_load(sc_ctx *c, const char *path, int32_t *n_applied) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!path) return fail(c, SC_EINVAL, "NULL path");
    FILE *f = fopen(path, "r");
    if (!f) return fail(c, SC_ENOTFOUND, "cannot read %s", path);
    int applied = 0;
    long long n, nnz, maxd;
    int k, B, inter, lmax, seg, wrow, t;
    double ms;
    while (fscanf(f, "%lld %lld %lld %d %d %d %d %d %d %d %lf", &n, &nnz, &maxd, &k, &B, &inter, &lmax, &seg, &wrow,
                  &t, &ms) == 11) {
        if (t < 1 || t > SC_MAX_T) break;
        std::vector<int32_t> e(2 * (t - 1));
        bool ok = true;
        for (auto &x : e) ok &= fscanf(f, "%d", &x) == 1;
        if (!ok) break;
        for (auto &gk : c->graphs)
            for (auto &tk : c->tmpls) {
                const Graph &g = *gk.second;
                if (g.n != n || g.nnz != nnz || g.max_deg != maxd || tk.second->edges != e) continue;
                Tuned tu;
                tu.interleave = inter;
                tu.lds_max = lmax;
                tu.seg = seg > 64 ? seg : 0;
                tu.wave_row_max = wrow >= 0 && wrow <= 40960 ? wrow : -1;
                tu.ms = ms;
                c->tuned[TuneKey{gk.first, tk.first, k, B}] = tu;
                ++applied;
            }
    }
    fclose(f);
    if (n_applied) *n_applied = applied;
    return SC_OK;
}

}  // extern "C"
