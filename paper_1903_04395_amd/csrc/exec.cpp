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

// Brackets one launch with HIP events on its stream while profiling is on.
struct ProfScope {
    sc_ctx *c;
    hipStream_t st;
    const char *name;
    double bytes, updates;
    hipEvent_t a = nullptr;
    ProfScope(sc_ctx *c_, bool on, hipStream_t st_, const char *n, double by, double up)
        : c(c_), st(st_), name(n), bytes(by), updates(up) {
        if (on && (a = next_event(c))) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = next_event(c);
        if (!b) return;
        (void)hipEventRecord(b, st);
        c->recs.push_back({name, a, b, bytes, updates});
    }
};

int ensure_gen(sc_ctx *c, DevMem &m, size_t bytes, hipStream_t st, PassBuffers &b) {
    if (m.p && m.bytes >= bytes) return SC_OK;
    uint64_t dummy = 0;
    int rc = ensure(c, m, bytes, st, &dummy);
    b.gen = g_buffer_generation.fetch_add(1);
    return rc;
}

size_t npre_bytes(const Graph &g, const Plan &P) {
    size_t w = 0;
    for (const Step &s : P.steps) w = std::max(w, (size_t)g.n_split * binom(P.k - 1, s.p) * P.batch);
    return w * 8;
}

// Kernel shape and device index tables of one step (tables are uploaded on
// first use, so prepare_pass calls this before any capture).
int step_args(sc_ctx *c, const Plan &P, const Step &s, uint64_t mod, kern::StepShape &sh,
              kern::StepTables &tb) {
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
    int rc;
    if (s.a > 1 && (rc = get_split(c, k - 1, s.h - 1, s.a - 1, &tb.split))) return rc;
    if (s.p > 1) {
        if ((rc = get_unrank(c, k - 1, s.p - 1, &tb.unrank))) return rc;
        if ((rc = get_rank(c, k - 1, &tb.rank))) return rc;
        tb.n_rank = kern::rank_entries(k - 1);
    }
    return SC_OK;
}

}  // namespace

int prepare_pass(sc_ctx *c, const PassSpec &s, PassBuffers &b, hipStream_t st) {
    Graph &g = *s.g;
    const Plan &P = *s.P;
    int rc;
    if ((rc = rebin(c, g, default_segment(c)))) return rc;
    if ((rc = ensure_gen(c, b.arena, P.arena_bytes, st, b))) return rc;
    if ((rc = ensure_gen(c, b.colbuf, (size_t)g.n_rows * P.batch, st, b))) return rc;
    if ((rc = ensure_gen(c, b.xbuf, (SC_MAX_BATCH + 1) * sizeof(uint64_t), st, b))) return rc;
    if ((rc = ensure_gen(c, b.desc, 2 * sizeof(uint64_t), st, b))) return rc;
    const size_t np = npre_bytes(g, P);
    if (np && (rc = ensure_gen(c, b.npre, np, st, b))) return rc;
    for (const Step &st_ : P.steps) {
        kern::StepShape sh;
        kern::StepTables tb;
        if ((rc = step_args(c, P, st_, s.mod, sh, tb))) return rc;
    }
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
    const double split_nnz = g.split_nnz, row_nnz = (double)g.nnz - split_nnz;

    HIPCHK(c, kern::launch_zero_u64((uint64_t *)X, SC_MAX_BATCH + 1, st));
    {
        ProfScope ps(c, prof, st, "color", dn * B, 0);
        HIPCHK(c, kern::launch_color((const uint64_t *)pb.desc.p, n, B, k, (const int32_t *)g.perm.p, col, st));
    }
    const Step *last = nullptr;
    for (const Step &s : P.steps) {
        kern::StepShape sh;
        kern::StepTables tb;
        if ((rc = step_args(c, P, s, sp.mod, sh, tb))) return rc;
        uint64_t *S = buf(s.buf_s);
        const uint64_t *Pp = buf(s.buf_p), *A = buf(s.buf_a);
        // updates in the paper's units (Lemma 1): nnz*C(k,p) neighbour-sum
        // updates, n*C(k,h)*C(h,a) multiply-adds (n*C(k,h) selects for a = 1)
        const double Wp = (double)binom(k, s.p), Wh = (double)binom(k, s.h);
        const double ema_upd = dn * Wh * (s.a > 1 ? (double)binom(s.h, s.a) : 1.0) * dB;
        if (g.n_split) {
            ProfScope ps(c, prof, st, "split", 4.0 * split_nnz + 16.0 * g.n_split * sh.Wn * dB,
                         split_nnz * Wp * dB);
            HIPCHK(c, kern::launch_dp_split(bins, sh, tb, col, Pp, Npre, flags, st));
        }
        // compulsory bytes: adjacency, colours, the passive and active tables
        // read once, the output written once, split rows' sums read back
        const double bytes = 4.0 * (double)g.nnz + 8.0 * (dn + 1) + dn * dB +
                             8.0 * dn * dB * ((s.p > 1 ? sh.Wq : 0) + (s.a > 1 ? sh.Wa : 0) + sh.Wh) +
                             8.0 * (double)g.n_split * sh.Wn * dB;
        ProfScope ps(c, prof, st, s.p == 1 ? "row_hist" : "row_gather", bytes, row_nnz * Wp * dB + ema_upd);
        HIPCHK(c, kern::launch_dp_row(bins, sh, tb, col, Pp, A, Npre, S, flags, st));
        last = &s;
    }
    const int W = (int)binom(k - 1, last->h - 1);
    ProfScope ps(c, prof, st, "reduce", 8.0 * dn * W * B, 0);
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
                         s.g->seg, s.mod, b.gen};
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

namespace {

constexpr size_t kStageWords = 2 + SC_MAX_BATCH + 1;   // descriptor + results of one pass

struct PassJob {
    int job, gid, tid, k;
    uint64_t seed, first;
    int offset;                // first colouring of this pass within its job
    uint64_t mod = 0;          // 0: uint64 counts with overflow flags; else residues mod this prime
    Plan P;
};

// Plans every pass of the jobs, runs them back to back on `st` and waits once.
int run_passes(sc_ctx *c, std::vector<PassJob> &passes, hipStream_t st,
               const std::function<void(const PassJob &, const uint64_t *)> &done) {
    int rc;
    if ((rc = host_staging(c, std::max<size_t>(1, passes.size()) * kStageWords))) return rc;
    // size the buffers for the largest pass first, so no buffer moves mid-chain
    size_t arena = 0, colb = 0, npre = 0;
    for (auto &p : passes) {
        const Graph &g = *c->graphs[p.gid];
        arena = std::max<size_t>(arena, p.P.arena_bytes);
        colb = std::max<size_t>(colb, (size_t)g.n_rows * p.P.batch);
        npre = std::max<size_t>(npre, npre_bytes(g, p.P));
    }
    PassBuffers &b = c->main;
    if ((rc = ensure_gen(c, b.arena, arena, st, b))) return rc;
    if ((rc = ensure_gen(c, b.colbuf, colb, st, b))) return rc;
    if (npre && (rc = ensure_gen(c, b.npre, npre, st, b))) return rc;
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

// Splits n colourings of one job into passes of the planned batch.
int plan_job(sc_ctx *c, int job, int gid, int tid, int k, uint64_t seed, uint64_t first, int n,
             std::vector<PassJob> &out) {
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

// ---------------------------------------------------------------- exact counts

// The three primes of the residue passes; with the uint64 pass they fix a count
// below their product times 2^64 (about 2^250).
constexpr uint64_t kPrimes[3] = {(1ull << 61) - 1, (1ull << 62) - 57, (1ull << 63) - 25};

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((unsigned __int128)a * b % p); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    for (a %= p; e; e >>= 1, a = mulmod(a, a, p))
        if (e & 1) r = mulmod(r, a, p);
    return r;
}

// x = x * m + add over nl little-endian limbs.
void big_muladd(uint64_t *x, int nl, uint64_t m, uint64_t add) {
    unsigned __int128 carry = add;
    for (int i = 0; i < nl; ++i) {
        const unsigned __int128 t = (unsigned __int128)x[i] * m + carry;
        x[i] = (uint64_t)t;
        carry = t >> 64;
    }
}

// The integer below 2^64 * p1 * ... * pm with residue r64 mod 2^64 and res[i]
// mod kPrimes[i], i < m <= 3 (Garner's mixed-radix form:
// x = v0 + 2^64 (v1 + p1 (v2 + p2 v3)), the digits of unused primes zero).
void crt_combine(uint64_t r64, const uint64_t res[3], int m, uint64_t out[4]) {
    uint64_t v[4] = {r64, 0, 0, 0};
    for (int i = 0; i < m; ++i) {
        const uint64_t p = kPrimes[i];
        // value of the digits so far mod p, and the radix (2^64 p1 .. p_{i-1}) mod p
        uint64_t acc = 0, radix = 1;
        for (int j = 0; j <= i; ++j) {
            acc = (acc + mulmod(v[j] % p, radix, p)) % p;
            radix = mulmod(radix, j == 0 ? (uint64_t)(((unsigned __int128)1 << 64) % p) : kPrimes[j - 1] % p, p);
        }
        const uint64_t diff = (res[i] % p + p - acc) % p;
        v[i + 1] = mulmod(diff, powmod(radix, p - 2, p), p);
    }
    uint64_t z[3] = {v[3], 0, 0};
    big_muladd(z, 3, kPrimes[1], v[2]);
    big_muladd(z, 3, kPrimes[0], v[1]);
    out[0] = v[0]; out[1] = z[0]; out[2] = z[1]; out[3] = z[2];
}

// Residues mod `mod` of colourings first..first+n-1.
int run_mod(sc_ctx *c, int gid, int tid, uint64_t first, int n, uint64_t mod, hipStream_t st, uint64_t *res) {
    std::vector<PassJob> passes;
    int rc = plan_job(c, 0, gid, tid, c->k, c->seed, first, n, passes);
    if (rc) return rc;
    for (auto &p : passes) p.mod = mod;
    return run_passes(c, passes, st, [&](const PassJob &p, const uint64_t *r) {
        for (int i = 0; i < p.P.batch; ++i) res[p.offset + i] = r[i] % mod;
    });
}

// Homomorphisms of the template into the graph, in double, by the plan's
// steps on one value per vertex (an upper bound on the colourful maps of any
// colouring).
int hom_count(sc_ctx *c, int gid, int tid, hipStream_t st, double *out) {
    Plan P;
    int rc = pick_batch(c, gid, tid, c->k, 1, 0, P);
    if (rc) return rc;
    Graph &g = *c->graphs[gid];
    if (P.steps.empty()) { *out = (double)g.n; return SC_OK; }
    if (g.n_rows == 0) { *out = 0; return SC_OK; }
    if ((rc = rebin(c, g, default_segment(c)))) return rc;
    const int64_t n = g.n_rows;
    DevMem tmp;
    if ((rc = dev_alloc(c, tmp, (P.bufs.size() * (size_t)n + 1) * sizeof(double)))) return rc;
    double *base = (double *)tmp.p;
    auto hb = [&](int id) { return id < 0 ? (double *)nullptr : base + 1 + (size_t)id * n; };
    const kern::GraphBins bins = bins_of(g);
    hipError_t e = kern::launch_zero_u64((uint64_t *)base, 1, st);
    const Step *last = nullptr;
    for (const Step &s : P.steps) {
        if (e != hipSuccess) break;
        e = kern::launch_hom_step(bins, hb(s.buf_a), hb(s.buf_p), hb(s.buf_s), st);
        last = &s;
    }
    if (e == hipSuccess) e = kern::launch_hom_sum(n, hb(last->buf_s), base, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, base, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(c, tmp);
    if (e != hipSuccess) return fail(c, SC_EDEVICE, "homomorphism count failed: %s", hipGetErrorString(e));
    return SC_OK;
}

// Counts below 2^kCrtBits[m-1] are fixed by their residues mod 2^64 and the
// first m primes (2^64 p1 > 2^124, 2^64 p1 p2 > 2^185, 2^64 p1 p2 p3 > 2^247).
constexpr int kCrtBits[3] = {124, 185, 247};

// Relative error of hom_count's double sums and products (t <= 32 rounded
// steps over at most 2^31 terms each, and the root sum) is far below this.
constexpr double kHomSlack = 1.0 + 0x1p-10;

// Residue primes a count bounded by H needs: the fewest that certify it, or
// all three (then only the residue mod their product is known).
int primes_for(double H) {
    for (int m = 1; m <= 3; ++m)
        if (H * kHomSlack < std::ldexp(1.0, kCrtBits[m - 1])) return m;
    return 3;
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

// Count of four little-endian limbs as a long double.
long double limbs_value(const uint64_t *l) {
    return (long double)l[0] + std::ldexp((long double)l[1], 64) + std::ldexp((long double)l[2], 128) +
           std::ldexp((long double)l[3], 192);
}

// Exact counts of colourings first..first+n-1 as four limbs each: the uint64
// pass, then residue passes for the colourings that overflowed, combined by
// CRT and certified by the homomorphism count (computed when a colouring
// overflowed or `want_hom`, into *H if that is still NaN).
int exact_counts(sc_ctx *c, int gid, int tid, uint64_t first, int ncol, hipStream_t st, uint64_t *counts,
                 uint8_t *exact, bool want_hom, double *H) {
    int rc;
    std::vector<uint64_t> c64((size_t)ncol);
    std::vector<uint8_t> ovf((size_t)ncol);
    {
        std::vector<PassJob> passes;
        if ((rc = plan_job(c, 0, gid, tid, c->k, c->seed, first, ncol, passes))) return rc;
        rc = run_passes(c, passes, st, [&](const PassJob &p, const uint64_t *res) {
            unpack_pass(res, p.P.batch, c64.data() + p.offset, ovf.data() + p.offset);
        });
        if (rc) return rc;
    }
    // the colourings that overflowed, in runs of consecutive ones, get residue
    // passes modulo as many primes as the homomorphism bound (every count is
    // at most the homomorphism count) asks for
    std::vector<std::pair<int, int>> runs;
    for (int r = 0; r < ncol; ++r) {
        if (!ovf[r]) continue;
        if (!runs.empty() && runs.back().first + runs.back().second == r) ++runs.back().second;
        else runs.push_back({r, 1});
    }
    if ((!runs.empty() || want_hom) && std::isnan(*H)) {
        if ((rc = hom_count(c, gid, tid, st, H))) return rc;
    }
    const int m = primes_for(*H);
    std::vector<uint64_t> res((size_t)3 * ncol);
    if (!runs.empty()) {
        std::vector<PassJob> passes;
        for (int i = 0; i < m; ++i)
            for (auto &ru : runs) {
                std::vector<PassJob> mine;
                if ((rc = plan_job(c, i, gid, tid, c->k, c->seed, first + (uint64_t)ru.first, ru.second, mine)))
                    return rc;
                for (auto &p : mine) {
                    p.mod = kPrimes[i];
                    p.offset += ru.first;
                    passes.push_back(std::move(p));
                }
            }
        rc = run_passes(c, passes, st, [&](const PassJob &p, const uint64_t *r) {
            for (int j = 0; j < p.P.batch; ++j) res[(size_t)p.job * ncol + p.offset + j] = r[j] % p.mod;
        });
        if (rc) return rc;
    }
    const bool certified = !runs.empty() && *H * kHomSlack < std::ldexp(1.0, kCrtBits[m - 1]);
    for (int r = 0; r < ncol; ++r) {
        uint64_t *out = counts + 4 * (size_t)r;
        if (!ovf[r]) {
            out[0] = c64[r]; out[1] = out[2] = out[3] = 0;
            exact[r] = 1;
        } else {
            const uint64_t rr[3] = {res[r], res[(size_t)ncol + r], res[2 * (size_t)ncol + r]};
            crt_combine(c64[r], rr, m, out);
            exact[r] = certified ? 1 : 0;
        }
    }
    return SC_OK;
}

// Colourings for an (eps, delta)-approximation of the count from i.i.d.
// colourings whose estimates have relative variance at most `relvar`: groups
// of g colourings make the group mean fail (miss by more than eps) with
// probability at most relvar / (g eps^2) <= 1/4 (Chebyshev), and the median of
// m groups fails only if half of them do, with probability at most
// exp(-m/8) <= delta (Hoeffding).  m is odd.
int colorings_for(int k, int t, double eps, double delta, double relvar, int32_t *m, int64_t *g) {
    if (!(eps > 0) || !(delta > 0) || !(delta < 1) || k < 1 || t < 1 || k < t || k > SC_MAX_K ||
        !(relvar >= 0))
        return SC_EINVAL;
    long double mm = std::ceil(8.0L * std::log(1.0L / (long double)delta));
    if (mm < 1) mm = 1;
    int32_t mi = (int32_t)std::min<long double>(mm, 1 << 30);
    if (mi % 2 == 0) ++mi;
    const long double gg = std::ceil(4.0L * (long double)relvar / ((long double)eps * eps));
    *m = mi;
    *g = (int64_t)std::max<long double>(1, std::min<long double>(gg, (long double)(INT64_MAX / 4) / mi));
    return SC_OK;
}

}  // namespace

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

int sc_run_mod(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, int32_t ncol, void *stream, uint64_t p,
               uint64_t *residues) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    int rc = check_run_args(c, gid, tid, ncol);
    if (rc) return rc;
    if (!kern::mod_supported(p)) return fail(c, SC_EINVAL, "modulus %llu is not 2^w - c (61 <= w <= 63, odd c <= 2^16)",
                                             (unsigned long long)p);
    if (ncol > 0 && !residues) return fail(c, SC_EINVAL, "NULL output");
    return run_mod(c, gid, tid, first, ncol, p, stream ? (hipStream_t)stream : c->stream, residues);
}

int sc_hom_count(sc_ctx *c, int32_t gid, int32_t tid, void *stream, double *out) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    int rc = check_run_args(c, gid, tid, 0);
    if (rc) return rc;
    if (!out) return fail(c, SC_EINVAL, "NULL output");
    return hom_count(c, gid, tid, stream ? (hipStream_t)stream : c->stream, out);
}

int sc_run_exact(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, int32_t ncol, void *stream,
                 uint64_t *counts, uint8_t *exact, double *hom_bound, double *est_maps, double *est_copies) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    int rc = check_run_args(c, gid, tid, ncol);
    if (rc) return rc;
    if (ncol > 0 && (!counts || !exact)) return fail(c, SC_EINVAL, "NULL output");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    double H = NAN;
    if ((rc = exact_counts(c, gid, tid, first, ncol, st, counts, exact, hom_bound != nullptr, &H))) return rc;
    if (hom_bound) *hom_bound = H;
    long double sum = 0;
    bool all = true;
    for (int r = 0; r < ncol; ++r) {
        all &= exact[r] != 0;
        sum += limbs_value(counts + 4 * (size_t)r);
    }
    const Template &T = *c->tmpls[tid];
    double m = NAN, cp = NAN;
    if (ncol > 0 && all) {
        m = (double)(sum / ncol) / colorful_probability(c->k, T.t);
        cp = m / T.aut;
    }
    if (est_maps) *est_maps = m;
    if (est_copies) *est_copies = cp;
    return SC_OK;
}

int sc_run_ablation(sc_ctx *c, int32_t gid, int32_t tid, int32_t variant, uint64_t first, int32_t ncol,
                    void *stream, uint64_t *counts, uint8_t *overflow) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    int rc = check_run_args(c, gid, tid, ncol);
    if (rc) return rc;
    if (variant != SC_ABL_FASCIA && variant != SC_ABL_PFASCIA) return fail(c, SC_EINVAL, "unknown variant %d", variant);
    if (ncol > 0 && (!counts || !overflow)) return fail(c, SC_EINVAL, "NULL output");
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    Plan P;
    if ((rc = pick_batch(c, gid, tid, c->k, 1, 0, P))) return rc;
    Graph &g = *c->graphs[gid];
    const int k = c->k;
    const int64_t n = g.n_rows;
    if (P.steps.empty() || n == 0) {
        for (int r = 0; r < ncol; ++r) { counts[r] = P.steps.empty() ? (uint64_t)g.n : 0; overflow[r] = 0; }
        return SC_OK;
    }
    if ((rc = rebin(c, g, default_segment(c)))) return rc;
    const kern::GraphBins bins = bins_of(g);
    // every table of the plan at once, in the paper's layout, plus the
    // neighbour sums (PFASCIA), the colours and the result words
    std::vector<DevMem> tabs(P.bufs.size());
    DevMem nbuf, colb, misc;
    auto release = [&]() {
        for (auto &m : tabs) dev_free(c, m);
        dev_free(c, nbuf); dev_free(c, colb); dev_free(c, misc);
    };
    int64_t wp_max = 0;
    for (const Step &s : P.steps) wp_max = std::max<int64_t>(wp_max, (int64_t)binom(k, s.p));
    for (size_t i = 0; i < P.bufs.size() && !rc; ++i)
        rc = dev_alloc(c, tabs[i], (size_t)n * binom(k, P.bufs[i].size) * 8);
    if (!rc && variant == SC_ABL_PFASCIA) rc = dev_alloc(c, nbuf, (size_t)n * wp_max * 8);
    if (!rc) rc = dev_alloc(c, colb, (size_t)n);
    if (!rc) rc = dev_alloc(c, misc, 4 * sizeof(uint64_t));
    if (rc) { release(); return rc; }
    auto tab = [&](int id) { return id < 0 ? (uint64_t *)nullptr : (uint64_t *)tabs[id].p; };
    auto *words = (uint64_t *)misc.p;            // desc[2], X, flag
    hipError_t e = hipSuccess;
    for (int r = 0; r < ncol && e == hipSuccess && !rc; ++r) {
        const uint64_t desc[2] = {c->seed, first + (uint64_t)r};
        e = hipMemcpyAsync(words, desc, sizeof(desc), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = kern::launch_zero_u64(words + 2, 2, st);
        if (e == hipSuccess)
            e = kern::launch_color(words, n, 1, k, (const int32_t *)g.perm.p, (uint8_t *)colb.p, st);
        const Step *last = nullptr;
        for (const Step &s : P.steps) {
            if (e != hipSuccess || rc) break;
            const uint32_t *split = nullptr;
            const uint16_t *pmask = nullptr;
            if ((rc = get_split(c, k, s.h, s.a, &split)) || (rc = get_unrank(c, k, s.p, &pmask))) break;
            e = kern::launch_ablation_step(variant, bins, k, s.a, s.p, (const uint8_t *)colb.p, split, pmask,
                                           tab(s.buf_a), tab(s.buf_p), (uint64_t *)nbuf.p, tab(s.buf_s),
                                           (unsigned long long *)(words + 3), st);
            last = &s;
        }
        if (e == hipSuccess && !rc)
            e = kern::launch_reduce(n, tab(last->buf_s), (int)binom(k, last->h), 1, 1, 0,
                                    (unsigned long long *)(words + 2), (unsigned long long *)(words + 3), st);
        uint64_t res[2] = {0, 0};
        if (e == hipSuccess && !rc) e = hipMemcpyAsync(res, words + 2, sizeof(res), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && !rc) e = hipStreamSynchronize(st);
        counts[r] = res[0];
        overflow[r] = res[1] ? 1 : 0;
    }
    if (e != hipSuccess) (void)hipStreamSynchronize(st);
    release();
    if (rc) return rc;
    if (e != hipSuccess) return fail(c, SC_EDEVICE, "ablation pass failed: %s", hipGetErrorString(e));
    return SC_OK;
}

int sc_colorings_for(int32_t k, int32_t t, double eps, double delta, int32_t *groups, int64_t *per_group) {
    if (!groups || !per_group) return SC_EINVAL;
    return colorings_for(k, t, eps, delta, 1.0 / colorful_probability(k, t) - 1.0, groups, per_group);
}

int sc_estimate(sc_ctx *c, int32_t gid, int32_t tid, uint64_t first, double eps, double delta, int32_t mode,
                int64_t max_colorings, void *stream, sc_estimate_t *out) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!out) return fail(c, SC_EINVAL, "NULL output");
    int rc = check_run_args(c, gid, tid, 0);
    if (rc) return rc;
    if (mode != SC_EST_BOUND && mode != SC_EST_SAMPLE) return fail(c, SC_EINVAL, "unknown mode %d", mode);
    const Template &T = *c->tmpls[tid];
    const double P = colorful_probability(c->k, T.t);
    int32_t m = 0;
    int64_t g = 0;
    if (colorings_for(c->k, T.t, eps, delta, 1.0 / P - 1.0, &m, &g))
        return fail(c, SC_EINVAL, "need 0 < eps and 0 < delta < 1 (eps=%g, delta=%g)", eps, delta);
    const int64_t cap = max_colorings > 0 ? max_colorings : INT64_MAX;
    if (cap < m) return fail(c, SC_EINVAL, "max_colorings=%lld is below the %d groups the median needs",
                             (long long)cap, m);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    std::vector<long double> y;                    // per colouring: count / P
    bool all = true;
    double H = NAN;
    auto run = [&](int64_t n) -> int {
        std::vector<uint64_t> limbs;
        std::vector<uint8_t> ex;
        while (n > 0) {
            const int chunk = (int)std::min<int64_t>(n, 1 << 20);
            limbs.assign(4 * (size_t)chunk, 0);
            ex.assign((size_t)chunk, 0);
            int r = exact_counts(c, gid, tid, first + (uint64_t)y.size(), chunk, st, limbs.data(), ex.data(), false, &H);
            if (r) return r;
            for (int i = 0; i < chunk; ++i) {
                all &= ex[i] != 0;
                y.push_back(limbs_value(limbs.data() + 4 * (size_t)i) / P);
            }
            n -= chunk;
        }
        return SC_OK;
    };
    int64_t need = (int64_t)m * g;                 // SC_EST_BOUND: the variance bound 1/P - 1
    if (mode == SC_EST_BOUND) {
        if (need > cap)
            return fail(c, SC_EINVAL, "the bound needs %lld colourings (%d groups of %lld), above max_colorings=%lld",
                        (long long)need, m, (long long)g, (long long)cap);
        if ((rc = run(need))) return rc;
    } else {
        // SC_EST_SAMPLE: the same rule with the sample relative variance, re-evaluated
        // after each round; rounds at most double the colourings run so far
        int64_t next = std::min<int64_t>(cap, 4 * (int64_t)m);
        for (;;) {
            if ((rc = run(next - (int64_t)y.size()))) return rc;
            long double mean = 0, var = 0;
            for (long double v : y) mean += v;
            mean /= (long double)y.size();
            for (long double v : y) var += (v - mean) * (v - mean);
            var /= (long double)(y.size() > 1 ? y.size() - 1 : 1);
            const double rel = mean > 0 ? (double)(var / (mean * mean)) : 0.0;
            int32_t m2 = 0;
            int64_t g2 = 0;
            colorings_for(c->k, T.t, eps, delta, rel, &m2, &g2);
            need = (int64_t)m2 * g2;
            if ((int64_t)y.size() >= need || (int64_t)y.size() >= cap) break;
            next = std::min<int64_t>({cap, need, 2 * (int64_t)y.size()});
        }
    }
    // median of the means of m groups of consecutive colourings
    const int64_t per = (int64_t)y.size() / m;
    std::vector<long double> means;
    for (int32_t i = 0; i < m && per > 0; ++i) {
        long double s = 0;
        for (int64_t j = 0; j < per; ++j) s += y[(size_t)(i * per + j)];
        means.push_back(s / per);
    }
    std::sort(means.begin(), means.end());
    long double mean_all = 0, var = 0;
    for (long double v : y) mean_all += v;
    mean_all /= (long double)std::max<size_t>(1, y.size());
    for (long double v : y) var += (v - mean_all) * (v - mean_all);
    var /= (long double)(y.size() > 1 ? y.size() - 1 : 1);
    out->colorings = (int64_t)y.size();
    out->groups = m;
    out->per_group = per;
    out->needed = need;
    out->exact = all ? 1 : 0;
    out->est_maps = means.empty() || !all ? NAN : (double)means[means.size() / 2];
    out->est_copies = out->est_maps / T.aut;
    out->mean_maps = all && !y.empty() ? (double)mean_all : NAN;
    out->rel_stderr = all && mean_all > 0 ? std::sqrt((double)(var / y.size())) / (double)mean_all : NAN;
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
    // interleave caps: the four largest powers of two dividing the batch
    std::vector<int> inter;
    for (int bi = 64; bi >= 1 && inter.size() < 4; bi /= 2)
        if (B % bi == 0) inter.push_back(bi);
    static const int ldss[] = {32 * 1024, 64 * 1024, 96 * 1024, 128 * 1024};
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    Tuned best;
    best.ms = 1e300;
    int trials = 0;
    for (int bi : inter)
        for (int lm : ldss) {
            Tuned cand;
            cand.interleave = bi;
            cand.lds_max = lm;
            c->tuned[key] = cand;
            std::vector<PassJob> passes;
            if ((rc = plan_job(c, 0, gid, tid, c->k, c->seed, 0, B, passes))) break;
            auto sink = [&](const PassJob &, const uint64_t *) {};
            if ((rc = run_passes(c, passes, c->stream, sink))) break;          // warm
            HIPCHK(c, hipEventRecord(e0, c->stream));
            if ((rc = run_passes(c, passes, c->stream, sink))) break;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            ++trials;
            if (ms < best.ms) { best = cand; best.ms = ms; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) { c->tuned.erase(key); return rc; }
    c->tuned[key] = best;
    out->interleave = best.interleave;
    out->lds_max = best.lds_max;
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
        fprintf(f, "%lld %lld %lld %d %d %d %d %d %.6f", (long long)g.n, (long long)g.nnz,
                (long long)g.max_deg, std::get<2>(kv.first), std::get<3>(kv.first),
                kv.second.interleave, kv.second.lds_max, T.t, kv.second.ms);
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
    int k, B, inter, lmax, t;
    double ms;
    while (fscanf(f, "%lld %lld %lld %d %d %d %d %d %lf", &n, &nnz, &maxd, &k, &B, &inter, &lmax, &t, &ms) == 9) {
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
