// libsc serving loop: resident graphs, continuously batched queries.
//
// A worker thread owns `max_inflight` slots, each a HIP stream with its own
// pass buffers.  Queries wait in FIFO order.  Whenever a slot is free, the
// query at the head gets a pass of as many of its colourings as fit the
// memory that is still free under the budget (so a large query runs in
// several passes, possibly on several slots at once, and a query that
// arrives while others run starts as soon as a slot and memory free up).
// Passes of different queries overlap on the device.  Completion is detected
// with events; results are unpacked into the query and the ticket becomes
// ready for sc_poll.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "rt.h"

namespace sc {

namespace {

// Streams of the serving loop: HIP maps a process's streams onto 4 hardware
// queues by default, so more streams only share them (and compete for the
// table budget).
constexpr int kMaxInflight = 4;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Query {
    uint64_t ticket = 0;
    sc_query_t q{};
    std::vector<uint64_t> counts;
    std::vector<uint8_t> ovf;
    int scheduled = 0, finished = 0;
    int status = SC_OK;
    double submit_s = 0, start_s = -1, done_s = -1;
    double est_maps = NAN, est_copies = NAN;
    bool done = false;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    PassBuffers buf;
    uint64_t *host = nullptr;     // pinned: descriptor (2 words) + results (SC_MAX_BATCH + 1)
    bool busy = false;
    Query *q = nullptr;
    Graph *g = nullptr;
    int offset = 0;
    Plan P;
};

struct ServeState {
    sc_serve_cfg_t cfg{};
    std::thread worker;
    std::mutex m;                                  // guards everything below but the slots
    std::condition_variable cv;
    std::deque<Query *> waiting;
    std::unordered_map<uint64_t, std::unique_ptr<Query>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;
    std::vector<Slot> slots;                       // worker thread only
    uint64_t passes = 0, colorings = 0, peak_bytes = 0, mem_bytes = 0;
    int inflight = 0;
};

namespace {

uint64_t slot_bytes(const Slot &s) {
    return s.buf.arena.bytes + s.buf.colbuf.bytes + s.buf.npre.bytes + s.buf.xbuf.bytes + s.buf.desc.bytes;
}

void finalize(sc_ctx *c, Query &Q) {
    Q.done = true;
    Q.done_s = now_s();
    if (Q.status) return;
    auto ti = c->tmpls.find(Q.q.tmpl_id);
    if (ti == c->tmpls.end()) return;
    bool any = false;
    double sum = 0;
    for (int i = 0; i < Q.q.n_colorings; ++i) { any |= Q.ovf[i] != 0; sum += (double)Q.counts[i]; }
    if (Q.q.n_colorings > 0 && !any) {
        Q.est_maps = sum / Q.q.n_colorings / colorful_probability(Q.q.k, ti->second->t);
        Q.est_copies = Q.est_maps / ti->second->aut;
    }
}

// Collects finished passes; returns whether any finished.
bool reap(sc_ctx *c, ServeState &S) {
    bool any = false;
    for (Slot &sl : S.slots) {
        if (!sl.busy) continue;
        hipError_t e = hipEventQuery(sl.ev);
        if (e == hipErrorNotReady) continue;
        any = true;
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        std::lock_guard<std::mutex> lq(S.m);
        Query &Q = *sl.q;
        if (e != hipSuccess) {
            Q.status = SC_EDEVICE;
            S.fatal = hipGetErrorString(e);
            for (auto it = S.waiting.begin(); it != S.waiting.end(); ++it)
                if (*it == &Q) { S.waiting.erase(it); break; }
        } else {
            unpack_pass(sl.host + 2, sl.P.batch, Q.counts.data() + sl.offset, Q.ovf.data() + sl.offset);
        }
        Q.finished += sl.P.batch;
        S.colorings += sl.P.batch;
        if ((Q.status && Q.finished >= Q.scheduled) || Q.finished >= Q.q.n_colorings) finalize(c, Q);
        sl.g->busy--;
        sl.busy = false;
        sl.q = nullptr;
        --S.inflight;
        S.cv.notify_all();
    }
    return any;
}

void fail_head(ServeState &S, Query &Q, int code) {
    Q.status = code;
    S.waiting.pop_front();
    if (Q.finished >= Q.scheduled) {
        Q.done = true;
        Q.done_s = now_s();
    }
    S.cv.notify_all();
}

// Starts passes on free slots; returns whether any started.
bool admit(sc_ctx *c, ServeState &S) {
    bool any = false;
    for (Slot &sl : S.slots) {
        if (sl.busy) continue;
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        Query *Q;
        {
            std::lock_guard<std::mutex> lq(S.m);
            if (S.waiting.empty()) return any;
            Q = S.waiting.front();
        }
        const int remaining = Q->q.n_colorings - Q->scheduled;
        const uint64_t others = S.mem_bytes - slot_bytes(sl);
        const uint64_t avail = S.cfg.mem_budget_bytes > others ? S.cfg.mem_budget_bytes - others : 0;
        Plan P;
        auto plan = [&](uint64_t budget) {
            return budget ? pick_batch(c, Q->q.graph_id, Q->q.tmpl_id, Q->q.k,
                                       std::min(remaining, S.cfg.max_batch), budget, P)
                          : SC_ENOMEM;
        };
        int rc = plan(avail);
        if (rc == SC_ENOMEM) {
            // give back what idle slots hold, then try once more
            for (Slot &o : S.slots)
                if (!o.busy && &o != &sl && slot_bytes(o)) {
                    (void)hipStreamSynchronize(o.st);
                    dev_free(c, o.buf.arena); dev_free(c, o.buf.colbuf); dev_free(c, o.buf.npre);
                    o.buf.gen = 0;
                }
            uint64_t mem = 0;
            for (const Slot &o : S.slots) mem += slot_bytes(o);
            {
                std::lock_guard<std::mutex> lq(S.m);
                S.mem_bytes = mem;
            }
            const uint64_t others2 = mem - slot_bytes(sl);
            rc = plan(S.cfg.mem_budget_bytes > others2 ? S.cfg.mem_budget_bytes - others2 : 0);
        }
        if (rc == SC_ENOMEM && S.inflight > 0) return any;   // wait for memory to free up
        if (rc) {
            std::lock_guard<std::mutex> lq(S.m);
            fail_head(S, *Q, rc);
            any = true;
            continue;
        }
        Graph *g = c->graphs[Q->q.graph_id].get();
        {
            // the plan fits what is left beside the other slots; this slot's
            // buffers only grow, so if keeping them would take the total past
            // the budget, release them first (the slot is idle)
            uint64_t mem = 0;
            for (const Slot &o : S.slots) mem += slot_bytes(o);
            const uint64_t others3 = mem - slot_bytes(sl);
            if (others3 + buffers_after(*g, P, sl.buf) > S.cfg.mem_budget_bytes) {
                (void)hipStreamSynchronize(sl.st);
                dev_free(c, sl.buf.arena); dev_free(c, sl.buf.colbuf); dev_free(c, sl.buf.npre);
                sl.buf.gen = 0;
            }
        }
        PassSpec spec;
        spec.g = g;
        spec.P = &sl.P;
        sl.P = std::move(P);
        spec.k = Q->q.k;
        spec.seed = Q->q.seed;
        spec.first = Q->q.first_coloring + (uint64_t)Q->scheduled;
        rc = launch_pass(c, Q->q.graph_id, Q->q.tmpl_id, spec, sl.buf, sl.st, sl.host, sl.host + 2,
                         c->use_graph != 0);
        if (!rc && hipEventRecord(sl.ev, sl.st) != hipSuccess) rc = SC_EDEVICE;
        uint64_t mem = 0;
        for (const Slot &o : S.slots) mem += slot_bytes(o);
        std::lock_guard<std::mutex> lq(S.m);
        S.mem_bytes = mem;
        S.peak_bytes = std::max(S.peak_bytes, mem);
        if (rc) {
            fail_head(S, *Q, rc);
            any = true;
            continue;
        }
        if (Q->start_s < 0) Q->start_s = now_s();
        sl.busy = true;
        sl.q = Q;
        sl.g = g;
        sl.offset = Q->scheduled;
        Q->scheduled += sl.P.batch;
        if (Q->scheduled >= Q->q.n_colorings) S.waiting.pop_front();
        g->busy++;
        ++S.inflight;
        ++S.passes;
        any = true;
    }
    return any;
}

void worker_loop(sc_ctx *c, ServeState *S) {
    (void)hipSetDevice(c->device);
    for (;;) {
        bool progressed = reap(c, *S);
        progressed |= admit(c, *S);
        std::unique_lock<std::mutex> lq(S->m);
        if (S->stop && S->waiting.empty() && S->inflight == 0) break;
        if (!progressed) {
            if (S->inflight > 0) {
                lq.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                S->cv.wait_for(lq, std::chrono::milliseconds(2));
            }
        }
    }
}

}  // namespace

void serve_shutdown(sc_ctx *c) {
    if (!c->serve) return;
    ServeState *S = c->serve;
    {
        std::lock_guard<std::mutex> lq(S->m);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (Slot &sl : S->slots) {
        (void)hipStreamSynchronize(sl.st);
        dev_free(c, sl.buf.arena); dev_free(c, sl.buf.colbuf); dev_free(c, sl.buf.xbuf);
        dev_free(c, sl.buf.npre); dev_free(c, sl.buf.desc);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (auto &kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
    c->graph_cache.clear();
    delete c->serve;
    c->serve = nullptr;
}

}  // namespace sc

using namespace sc;

extern "C" {

int sc_serve_start(sc_ctx *c, const sc_serve_cfg_t *cfg) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!cfg) return fail(c, SC_EINVAL, "NULL config");
    if (c->serve) return fail(c, SC_ESTATE, "the serving loop already runs");
    if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxInflight)
        return fail(c, SC_EINVAL, "max_inflight must be in [1, %d]", kMaxInflight);
    if (cfg->max_batch < 1 || cfg->max_batch > SC_MAX_BATCH) return fail(c, SC_EINVAL, "max_batch must be in [1, %d]", SC_MAX_BATCH);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_EDEVICE, "hipSetDevice failed");
    // the count tables of the synchronous calls would hold device memory
    // beside the serving budget: give them back (a later sc_run regrows them)
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dev_free(c, c->main.arena); dev_free(c, c->main.colbuf); dev_free(c, c->main.npre);
    c->main.gen = 0;
    auto S = std::make_unique<ServeState>();
    S->cfg = *cfg;
    if (!S->cfg.mem_budget_bytes) S->cfg.mem_budget_bytes = c->budget;
    S->slots.resize(cfg->max_inflight);
    for (Slot &sl : S->slots) {
        void *p = nullptr;
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&p, (3 + SC_MAX_BATCH) * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
            c->serve = S.release();
            serve_shutdown(c);
            return fail(c, SC_EDEVICE, "cannot create the serving streams");
        }
        sl.host = (uint64_t *)p;
    }
    ServeState *raw = S.release();
    c->serve = raw;
    raw->worker = std::thread(worker_loop, c, raw);
    return SC_OK;
}

int sc_submit(sc_ctx *c, const sc_query_t *q, uint64_t *ticket) {
    if (!c) return SC_EINVAL;
    if (!q || !ticket) return fail(c, SC_EINVAL, "NULL argument");
    {
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (!c->serve) return fail(c, SC_ESTATE, "the serving loop is not running");
        auto gi = c->graphs.find(q->graph_id);
        if (gi == c->graphs.end()) return fail(c, SC_ENOTFOUND, "unknown graph %d", q->graph_id);
        auto ti = c->tmpls.find(q->tmpl_id);
        if (ti == c->tmpls.end()) return fail(c, SC_ENOTFOUND, "unknown template %d", q->tmpl_id);
        if (q->k < ti->second->t || q->k > SC_MAX_K) return fail(c, SC_EINVAL, "need t <= k <= 16");
        if (q->n_colorings < 1) return fail(c, SC_EINVAL, "n_colorings must be >= 1");
        if (int rc = check_coloring_range(c, q->first_coloring, q->n_colorings)) return rc;
    }
    ServeState &S = *c->serve;
    auto Q = std::make_unique<Query>();
    Q->q = *q;
    Q->counts.assign(q->n_colorings, 0);
    Q->ovf.assign(q->n_colorings, 0);
    Q->submit_s = now_s();
    {
        std::lock_guard<std::mutex> lq(S.m);
        if (S.stop) return fail(c, SC_ESTATE, "the serving loop is stopping");
        Q->ticket = S.next_ticket++;
        *ticket = Q->ticket;
        S.waiting.push_back(Q.get());
        S.all[Q->ticket] = std::move(Q);
    }
    S.cv.notify_all();
    return SC_OK;
}

int sc_poll(sc_ctx *c, uint64_t ticket, sc_result_t *out) {
    if (!c) return SC_EINVAL;
    if (!out) return fail(c, SC_EINVAL, "NULL argument");
    if (!c->serve) return fail(c, SC_ESTATE, "the serving loop is not running");
    ServeState &S = *c->serve;
    std::lock_guard<std::mutex> lq(S.m);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return SC_ENOTFOUND;
    Query &Q = *it->second;
    if (!Q.done) return SC_EBUSY;
    out->status = Q.status;
    out->n_colorings = Q.q.n_colorings;
    if (out->counts) std::copy(Q.counts.begin(), Q.counts.end(), out->counts);
    if (out->overflow) std::copy(Q.ovf.begin(), Q.ovf.end(), out->overflow);
    out->est_maps = Q.est_maps;
    out->est_copies = Q.est_copies;
    out->submit_s = Q.submit_s;
    out->start_s = Q.start_s;
    out->done_s = Q.done_s;
    S.all.erase(it);
    return SC_OK;
}

int sc_serve_stats(sc_ctx *c, sc_serve_stats_t *out) {
    if (!c || !out) return SC_EINVAL;
    if (!c->serve) return fail(c, SC_ESTATE, "the serving loop is not running");
    ServeState &S = *c->serve;
    std::lock_guard<std::mutex> lq(S.m);
    out->passes = S.passes;
    out->colorings = S.colorings;
    out->waiting = (int32_t)S.waiting.size();
    out->inflight = S.inflight;
    out->mem_bytes = S.mem_bytes;
    out->peak_mem_bytes = S.peak_bytes;
    return SC_OK;
}

int sc_serve_stop(sc_ctx *c) {
    if (!c) return SC_EINVAL;
    if (!c->serve) return fail(c, SC_ESTATE, "the serving loop is not running");
    serve_shutdown(c);
    return SC_OK;
}

}  // extern "C"
