// sc_run_static: sc_run for callers that cannot allocate device memory.
//
// Every buffer of a pass -- the colouring descriptor, the result words, the
// index tables, the colours, the split rows' neighbour sums and the count
// tables -- lives in one file-scope device array of SC_STATIC_SCRATCH_BYTES.
// Each device the library runs on holds its own copy of the array (in every
// process that loads the library) until the process ends.  The host never
// names the array directly: its device address comes from
// hipGetSymbolAddress, taken once per device when a context is created there.
// The kernels are the ones sc_run launches; only where their buffers live
// differs.
#include <hip/hip_runtime.h>

#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "rt.h"

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[SC_STATIC_SCRATCH_BYTES];

std::mutex g_init_mu;
void *g_scratch_ptr[kMaxDevices];     // device address of `scratch` on each device (null: not set up)
std::mutex g_run_mu[kMaxDevices];     // one allocation-free call per device at a time

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Where one pass's buffers sit in the scratch array, and the host copies of
// its index tables (kept until the call has waited for its stream).
struct StaticPass {
    size_t desc = 0, xbuf = 0, col = 0, npre = 0, arena = 0, total = 0;
    struct Tab {
        size_t off;
        std::vector<uint8_t> bytes;
    };
    std::vector<Tab> tabs;
    sc::StagedTables staged;
};

template <typename T>
void add_table(StaticPass &L, size_t &off, std::vector<T> v) {
    StaticPass::Tab t;
    t.off = off;
    t.bytes.resize(v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(t.bytes.data(), v.data(), t.bytes.size());
    off = align_up(off + std::max<size_t>(t.bytes.size(), 1));
    L.tabs.push_back(std::move(t));
}

// Lays out a pass of plan P on graph g from offset 0 of the scratch array,
// with device pointers into `base` for the staged tables.
void layout_pass(const sc::Graph &g, const sc::Plan &P, unsigned char *base, StaticPass &L) {
    using sc::TableKey;
    const int k = P.k;
    size_t off = 0;
    L.desc = off;  off = align_up(off + 2 * sizeof(uint64_t));
    L.xbuf = off;  off = align_up(off + (SC_MAX_BATCH + 1) * sizeof(uint64_t));
    auto stage_unrank = [&](int sz) {
        const TableKey ukey{k - 1, sz, 0};
        if (!L.staged.unrank.count(ukey)) {
            L.staged.unrank[ukey] = (const uint16_t *)(base + off);
            add_table(L, off, sc::unrank_table(k - 1, sz));
        }
    };
    auto stage_rank = [&]() {
        const TableKey rkey{k - 1, 0, 0};
        if (!L.staged.rank.count(rkey)) {
            L.staged.rank[rkey] = (const uint16_t *)(base + off);
            add_table(L, off, sc::rank_table(k - 1));
        }
    };
    for (const sc::Step &s : P.steps) {
        if (s.a > 1) {
            const TableKey key{k - 1, s.h - 1, s.a - 1};
            if (!L.staged.split.count(key)) {
                L.staged.split[key] = (const uint32_t *)(base + off);
                add_table(L, off, sc::split_table(k - 1, s.h - 1, s.a - 1));
            }
        }
        if (s.p > 1) {
            stage_unrank(s.p - 1);
            stage_rank();
        }
    }
    L.col = off;   off = align_up(off + (size_t)g.n_rows * P.batch);
    L.npre = off;  off = align_up(off + sc::npre_bytes(g, P));
    L.arena = off; off = align_up(off + P.arena_bytes);
    L.total = off;
}

sc::DevMem view(unsigned char *base, size_t off, size_t bytes) {
    sc::DevMem m;
    m.p = base + off;
    m.bytes = bytes;
    return m;
}

}  // namespace

namespace sc {

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SC_EINVAL;
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_scratch_ptr[device]) return SC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return SC_EDEVICE;
    }
    g_scratch_ptr[device] = p;
    return SC_OK;
}

}  // namespace sc

using namespace sc;

extern "C" int sc_run_static(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, int32_t ncol, void *stream,
                             uint64_t *counts, uint8_t *overflow, double *est_maps, double *est_copies) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (ncol < 0) return fail(c, SC_EINVAL, "n_colorings < 0");
    if (ncol > 0 && (!counts || !overflow)) return fail(c, SC_EINVAL, "NULL output");
    if (int rc = check_run_args(c, gid, tid, ncol)) return rc;
    if (int rc = check_coloring_range(c, first, ncol)) return rc;
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, SC_EDEVICE, "device %d out of range", c->device);
    unsigned char *base = (unsigned char *)g_scratch_ptr[c->device];
    if (!base) return fail(c, SC_EDEVICE, "the static scratch of device %d is not set up", c->device);
    Graph &g = *c->graphs[gid];
    const Template &T = *c->tmpls[tid];
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    const int k = c->k;

    // passes: the largest batch (in pick_batch's order) whose buffers fit the array
    struct Pass {
        Plan P;
        uint64_t first;
        int offset;
        StaticPass L;
        uint64_t desc[2];
        uint64_t res[SC_MAX_BATCH + 1];
    };
    std::list<Pass> passes;   // stable addresses: the host copies are read by the stream
    int off = 0;
    while (off < ncol) {
        const int want = std::max(1, std::min<int>(ncol - off, (int)std::min<int64_t>(c->max_batch, SC_MAX_BATCH)));
        Pass ps;
        bool fits = false;
        for (int b = want; b >= 1;) {
            const ExecOpts o = exec_opts(c, gid, tid, k, b);
            if (int rc = make_plan(c, g, T, o, k, b, ps.P)) return rc;
            ps.L = StaticPass{};
            layout_pass(g, ps.P, base, ps.L);
            if (ps.L.total <= SC_STATIC_SCRATCH_BYTES) { fits = true; break; }
            if (b > 8) b = b % 8 ? b - b % 8 : b - 8;
            else b = b > 4 ? 4 : b / 2;
        }
        if (!fits)
            return fail(c, SC_ENOMEM, "one colouring needs %zu bytes of device buffers; the static scratch holds %llu",
                        ps.L.total, (unsigned long long)SC_STATIC_SCRATCH_BYTES);
        // the heavy-row bins of the plan's segment size must exist already
        // (switching to them allocates nothing; building them would)
        const int seg = plan_segment(c, ps.P);
        if (seg != g.seg && !g.saved_bins.count(seg))
            return fail(c, SC_ESTATE, "graph %d has no heavy-row bins for segment size %d (the allocation-free "
                        "run cannot build them; run sc_run once with this segment size)", gid, seg);
        ps.first = first + (uint64_t)off;
        ps.offset = off;
        off += ps.P.batch;
        passes.push_back(std::move(ps));
    }

    std::lock_guard<std::mutex> run_lk(g_run_mu[c->device]);
    // on an error, wait for what was enqueued: copies into the host buffers
    // above may still be in flight
    auto failed = [&](int rc) {
        (void)hipStreamSynchronize(st);
        return rc;
    };
#define SC_STATIC_CHK(expr)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return failed(fail(c, SC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)));  \
    } while (0)
    for (Pass &ps : passes) {
        const Plan &P = ps.P;
        if (P.steps.empty() || g.n_rows == 0) {      // t = 1: every vertex is a map; no edge: no map
            for (int r = 0; r < SC_MAX_BATCH; ++r) ps.res[r] = P.steps.empty() ? (uint64_t)g.n : 0;
            ps.res[SC_MAX_BATCH] = 0;
            continue;
        }
        for (const auto &t : ps.L.tabs)
            if (!t.bytes.empty())
                SC_STATIC_CHK(hipMemcpyAsync(base + t.off, t.bytes.data(), t.bytes.size(), hipMemcpyHostToDevice, st));
        if (int rc = rebin(c, g, plan_segment(c, P), false)) return failed(rc);
        ps.desc[0] = c->seed;
        ps.desc[1] = ps.first;
        SC_STATIC_CHK(hipMemcpyAsync(base + ps.L.desc, ps.desc, sizeof ps.desc, hipMemcpyHostToDevice, st));
        PassBuffers pb;
        pb.desc = view(base, ps.L.desc, 2 * sizeof(uint64_t));
        pb.xbuf = view(base, ps.L.xbuf, (SC_MAX_BATCH + 1) * sizeof(uint64_t));
        pb.colbuf = view(base, ps.L.col, (size_t)g.n_rows * P.batch);
        pb.npre = view(base, ps.L.npre, npre_bytes(g, P));
        pb.arena = view(base, ps.L.arena, P.arena_bytes);
        pb.staged = &ps.L.staged;
        PassSpec spec;
        spec.g = &g;
        spec.P = &P;
        spec.k = k;
        spec.seed = c->seed;
        spec.first = ps.first;
        if (int rc = enqueue_pass(c, spec, pb, st, false)) return failed(rc);
        SC_STATIC_CHK(hipMemcpyAsync(ps.res, pb.xbuf.p, sizeof ps.res, hipMemcpyDeviceToHost, st));
    }
#undef SC_STATIC_CHK
    HIPCHK(c, hipStreamSynchronize(st));
    for (const Pass &ps : passes) unpack_pass(ps.res, ps.P.batch, counts + ps.offset, overflow + ps.offset);
    estimates(counts, overflow, ncol, k, T.t, T.aut, est_maps, est_copies);
    return SC_OK;
}
