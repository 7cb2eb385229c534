// libsc host side of the pruning-ablation baselines (FASCIA, PFASCIA): every
// table of the plan in the paper's layout, one colouring at a time through
// the plain kernels of ablation.hip.
#include <algorithm>
#include <vector>

#include "rt.h"

using namespace sc;

extern "C" {

int sc_run_ablation(sc_ctx *c, int32_t gid, int32_t tid, int32_t variant, uint64_t first, int32_t ncol,
                    void *stream, uint64_t *counts, uint8_t *overflow) {
    if (!c) return SC_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    int rc = check_run_args(c, gid, tid, ncol);
    if (!rc) rc = check_coloring_range(c, first, ncol);
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
        rc = dev_alloc(c, tabs[i], (size_t)n * binom(k, P.bufs[i].size) * 8, st);
    if (!rc && variant == SC_ABL_PFASCIA) rc = dev_alloc(c, nbuf, (size_t)n * wp_max * 8, st);
    if (!rc) rc = dev_alloc(c, colb, (size_t)n, st);
    if (!rc) rc = dev_alloc(c, misc, 4 * sizeof(uint64_t), st);
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

}  // extern "C"
