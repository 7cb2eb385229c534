// libsc exact wide counts and the (eps, delta) estimator: residue passes
// modulo primes of the form 2^w - c, their combination with the uint64 pass by
// the Chinese remainder theorem, the homomorphism-count bound that picks the
// primes and certifies the result, and the median-of-means estimate over
// exact counts.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "rt.h"

using namespace sc;

namespace {

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
// colouring).  step_max (optional): per step of the plan, its (h, a, p) and
// the largest value at any vertex (a bound on every entry of that step's
// table in any colouring).
struct StepBound {
    int h, a, p;
    double max;
};
int hom_count(sc_ctx *c, int gid, int tid, hipStream_t st, double *out, std::vector<StepBound> *step_max = nullptr) {
    Plan P;
    int rc = pick_batch(c, gid, tid, c->k, 1, 0, P);
    if (rc) return rc;
    Graph &g = *c->graphs[gid];
    if (step_max) step_max->clear();
    if (P.steps.empty()) { *out = (double)g.n; return SC_OK; }
    if (g.n_rows == 0) { *out = 0; return SC_OK; }
    if ((rc = rebin(c, g, default_segment(c)))) return rc;
    const int64_t n = g.n_rows;
    const size_t ns = P.steps.size(), head = 1 + ns;       // the sum, then the step maxima
    DevMem tmp;
    if ((rc = dev_alloc(c, tmp, (P.bufs.size() * (size_t)n + head) * sizeof(double), st))) return rc;
    double *base = (double *)tmp.p;
    auto hb = [&](int id) { return id < 0 ? (double *)nullptr : base + head + (size_t)id * n; };
    const kern::GraphBins bins = bins_of(g);
    hipError_t e = kern::launch_zero_u64((uint64_t *)base, (int64_t)head, st);
    const Step *last = nullptr;
    for (size_t i = 0; i < ns; ++i) {
        const Step &s = P.steps[i];
        if (e == hipSuccess) e = kern::launch_hom_step(bins, hb(s.buf_a), hb(s.buf_p), hb(s.buf_s), st);
        if (e == hipSuccess && step_max) e = kern::launch_hom_max(n, hb(s.buf_s), base + 1 + i, st);
        last = &s;
    }
    std::vector<double> host(head);
    if (e == hipSuccess) e = kern::launch_hom_sum(n, hb(last->buf_s), base, st);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), base, head * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(c, tmp);
    if (e == hipSuccess) {
        *out = host[0];
        if (step_max)
            for (size_t i = 0; i < ns; ++i)
                step_max->push_back({P.steps[i].h, P.steps[i].a, P.steps[i].p, host[1 + i]});
    }
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


// Limbs of 64 bits that hold every value up to the bound x (with the
// homomorphism count's margin); 5 if four do not.
int limbs_for(double x) {
    int l = 1;
    while (l <= 4 && !(x * kHomSlack < std::ldexp(1.0, 64 * l))) ++l;
    return l;
}

// Per step of a single-chain plan, the limbs its entries keep in the exact
// multi-limb pass: step i's bound (the largest homomorphism count of its
// sub-template at any vertex), never fewer than the step before, the colour
// counts of step 0 in one, and the last step at least what the total bound H
// asks for, so that the root sums fit.  Empty when that pass does not apply:
// H below 2^64 (the uint64 pass is exact), a bound past four limbs, rows too
// wide for the LDS limit, or bounds that do not match the plan's steps.
std::vector<int> chain_limbs(double H, const std::vector<StepBound> &bounds, const std::vector<PassJob> &passes) {
    const int total = limbs_for(H);
    if (total < 2 || total > 4 || passes.empty()) return {};
    const Plan &P = passes[0].P;
    if (bounds.size() != P.steps.size()) return {};
    std::vector<int> limbs(P.steps.size());
    for (size_t i = 0; i < limbs.size(); ++i) {
        const Step &s = P.steps[i];
        if (bounds[i].h != s.h || bounds[i].a != s.a || bounds[i].p != s.p) return {};
        limbs[i] = i == 0 ? 1 : std::max(limbs[i - 1], limbs_for(bounds[i].max));
        if (limbs[i] > 4) return {};
    }
    limbs.back() = std::max(limbs.back(), total);
    for (const PassJob &p : passes) {
        if (p.P.steps.size() != limbs.size()) return {};
        int wrow = 0;                       // the widest intermediate row, in words per colouring
        for (size_t i = 1; i + 1 < limbs.size(); ++i)
            wrow = std::max(wrow, (int)binom(p.k - 1, p.P.steps[i].h - 1) * limbs[i]);
        if (kern::chain_wide_lds_bytes(p.k - 1, wrow, 1) > p.P.opts.lds_max) return {};
    }
    return limbs;
}

// Count of four little-endian limbs as a long double.
long double limbs_value(const uint64_t *l) {
    return (long double)l[0] + std::ldexp((long double)l[1], 64) + std::ldexp((long double)l[2], 128) +
           std::ldexp((long double)l[3], 192);
}

// Exact counts of colourings first..first+n-1 as four limbs each.  A
// single-chain template whose homomorphism bound passes 2^64 takes one
// multi-limb pass.  Otherwise the uint64
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
        // a template that is one chain from a single vertex (a star rooted at
        // its centre) whose counts may pass 2^64 runs once with as many
        // 64-bit limbs as the homomorphism bound asks for
        bool chains = !passes.empty();
        for (const PassJob &p : passes) chains &= single_chain(p.P);
        std::vector<StepBound> bounds;
        if (chains && (rc = hom_count(c, gid, tid, st, H, &bounds))) return rc;
        const std::vector<int> limbs = chains ? chain_limbs(*H, bounds, passes) : std::vector<int>();
        if (!limbs.empty()) {
            const int L = limbs.back();
            std::vector<uint8_t> bad((size_t)ncol);
            rc = run_wide_passes(c, passes, limbs, st, [&](const PassJob &p, const uint64_t *x, uint64_t flags) {
                for (int i = 0; i < p.P.batch; ++i) {
                    uint64_t *out = counts + 4 * (size_t)(p.offset + i);
                    const uint64_t *xi = x + (size_t)i * (L + 1);
                    for (int l = 0; l < 4; ++l) out[l] = l < L ? xi[l] : 0;
                    bad[p.offset + i] = ((flags >> i) & 1) || xi[L] != 0;
                }
            });
            if (rc) return rc;
            for (int r = 0; r < ncol; ++r) exact[r] = bad[r] ? 0 : 1;
            return SC_OK;
        }
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
        if ((rc = check_coloring_range(c, first, need))) return rc;
        if (need > cap)
            return fail(c, SC_EINVAL, "the bound needs %lld colourings (%d groups of %lld), above max_colorings=%lld",
                        (long long)need, m, (long long)g, (long long)cap);
        if ((rc = run(need))) return rc;
    } else {
        // SC_EST_SAMPLE: the same rule with the sample relative variance, re-evaluated
        // after each round; rounds at most double the colourings run so far
        int64_t next = std::min<int64_t>(cap, 4 * (int64_t)m);
        for (;;) {
            if ((rc = check_coloring_range(c, first, next))) return rc;
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

}  // extern "C"
