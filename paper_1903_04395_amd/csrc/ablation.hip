// Plain kernels of the two CPU designs the paper improves on, kept as
// baselines for its pruning ablation (Sec. 3.1, Sec. 4.1, Sec. 7.1): one
// colouring at a time, tables in the paper's layout (row v of sub-template
// size s holds all binom(k, s) colour sets, column = Eq. 1 rank), one thread
// per table entry.
//
//  * FASCIA (Algorithm 1): for every row, output set and split, the passive
//    child's column is summed over the row's neighbours again -- the redundant
//    neighbour traversal of Sec. 3.1.
//  * PFASCIA (pruned, Sec. 4.1): the neighbour sum of every passive column is
//    taken once per row, then the split multiply-add reads it.
//
// Counts are exact uint64 with the library's overflow rule: a neighbour sum
// counts only where its set leaves out the row's own colour, products and
// table entries always, the root sum always.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "exact.h"      // after the HIP runtime header (it uses __device__)

namespace sc {
namespace kern {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kGridCap = 1 << 16;

struct AblArgs {
    const int64_t *rp;
    const int32_t *ci;
    const uint8_t *col;                 // colour of every row (one colouring)
    int64_t n;
    int a, p;                           // sizes of the active and passive children
    int Wa, Wp, Wh, nsplit;             // binom(k, a), binom(k, p), binom(k, h), binom(h, a)
    const uint32_t *split;              // (k, h, a) split table: per output set, nsplit (Ia | Ip << 16)
    const uint16_t *pmask;              // colour masks of the p-subsets of k colours, in rank order
    const uint64_t *A, *P;              // tables of the children (NULL: single vertex)
    uint64_t *N;                        // PFASCIA: neighbour sums [n][Wp]
    uint64_t *S;
    unsigned long long *flag;
};

// Entry of the single-vertex table: the set {c} has rank c.
__device__ __forceinline__ uint64_t leaf_entry(const uint8_t *col, int64_t v, int I) {
    return col[v] == I ? 1u : 0u;
}

// Sum over the neighbours of v of column Ip of the passive table; sets `ovf`
// on a carry.
__device__ __forceinline__ uint64_t neighbour_sum(const AblArgs &a, int64_t v, int Ip, uint32_t &ovf) {
    uint64_t y = 0;
    for (int64_t e = a.rp[v]; e < a.rp[v + 1]; ++e) {
        const int64_t u = a.ci[e];
        const uint64_t x = a.P ? a.P[u * a.Wp + Ip] : leaf_entry(a.col, u, Ip);
        y += x;
        ovf |= (uint32_t)(y < x);
    }
    return y;
}

__global__ __launch_bounds__(kThreads) void fascia_step_kernel(AblArgs a) {
    uint32_t bad = 0;
    const int64_t total = a.n * a.Wh;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += (int64_t)gridDim.x * kThreads) {
        const int64_t v = q / a.Wh;
        const int Is = (int)(q - v * a.Wh);
        const uint32_t *sp = a.split + Is;                 // pair j at sp[j * Wh]
        uint64_t acc = 0;
        uint32_t ovf = 0;
        for (int j = 0; j < a.nsplit; ++j) {
            const uint32_t pr = sp[(int64_t)j * a.Wh];
            const int Ia = (int)(pr & 0xffffu), Ip = (int)(pr >> 16);
            const uint64_t x = a.A ? a.A[v * a.Wa + Ia] : leaf_entry(a.col, v, Ia);
            uint32_t novf = 0;
            const uint64_t y = neighbour_sum(a, v, Ip, novf);      // again for every split
            if (!((a.pmask[Ip] >> a.col[v]) & 1u)) ovf |= novf;
            acc = mad_ovf(acc, x, y, ovf);
        }
        a.S[q] = acc;
        bad |= ovf;
    }
    if (__any(bad)) {
        if ((threadIdx.x & 63) == 0) atomicOr(a.flag, 1ull);
    }
}

__global__ __launch_bounds__(kThreads) void pfascia_sum_kernel(AblArgs a) {
    uint32_t bad = 0;
    const int64_t total = a.n * a.Wp;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += (int64_t)gridDim.x * kThreads) {
        const int64_t v = q / a.Wp;
        const int Ip = (int)(q - v * a.Wp);
        uint32_t ovf = 0;
        a.N[q] = neighbour_sum(a, v, Ip, ovf);
        if (!((a.pmask[Ip] >> a.col[v]) & 1u)) bad |= ovf;
    }
    if (__any(bad)) {
        if ((threadIdx.x & 63) == 0) atomicOr(a.flag, 1ull);
    }
}

__global__ __launch_bounds__(kThreads) void pfascia_ema_kernel(AblArgs a) {
    uint32_t bad = 0;
    const int64_t total = a.n * a.Wh;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += (int64_t)gridDim.x * kThreads) {
        const int64_t v = q / a.Wh;
        const int Is = (int)(q - v * a.Wh);
        const uint32_t *sp = a.split + Is;                 // pair j at sp[j * Wh]
        uint64_t acc = 0;
        uint32_t ovf = 0;
        for (int j = 0; j < a.nsplit; ++j) {
            const uint32_t pr = sp[(int64_t)j * a.Wh];
            const int Ia = (int)(pr & 0xffffu), Ip = (int)(pr >> 16);
            const uint64_t x = a.A ? a.A[v * a.Wa + Ia] : leaf_entry(a.col, v, Ia);
            acc = mad_ovf(acc, x, a.N[v * a.Wp + Ip], ovf);
        }
        a.S[q] = acc;
        bad |= ovf;
    }
    if (__any(bad)) {
        if ((threadIdx.x & 63) == 0) atomicOr(a.flag, 1ull);
    }
}

unsigned grid_for(int64_t total) {
    const int64_t b = (total + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : (b > kGridCap ? kGridCap : b));
}

}  // namespace

hipError_t launch_ablation_step(int variant, const GraphBins &g, int k, int a, int p, const uint8_t *col,
                                const uint32_t *split, const uint16_t *pmask, const uint64_t *A,
                                const uint64_t *P, uint64_t *N, uint64_t *S, unsigned long long *flag,
                                hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    auto binom = [](int n, int r) {
        if (r < 0 || r > n) return (int64_t)0;
        int64_t b = 1;
        for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i;
        return b;
    };
    const int h = a + p;
    if (a < 1 || p < 1 || h > k || k > 16 || !split || !pmask || !S || !flag || (a > 1 && !A) ||
        (p > 1 && !P) || (variant == kAblPfascia && !N) || (variant != kAblFascia && variant != kAblPfascia))
        return hipErrorInvalidValue;
    AblArgs x{};
    x.rp = g.row_ptr; x.ci = g.col_idx; x.col = col; x.n = g.n;
    x.a = a; x.p = p;
    x.Wa = (int)binom(k, a); x.Wp = (int)binom(k, p); x.Wh = (int)binom(k, h); x.nsplit = (int)binom(h, a);
    x.split = split; x.pmask = pmask;
    x.A = a > 1 ? A : nullptr;
    x.P = p > 1 ? P : nullptr;
    x.N = N; x.S = S; x.flag = flag;
    if (variant == kAblFascia) {
        fascia_step_kernel<<<grid_for(g.n * x.Wh), kThreads, 0, st>>>(x);
        return hipGetLastError();
    }
    pfascia_sum_kernel<<<grid_for(g.n * x.Wp), kThreads, 0, st>>>(x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    pfascia_ema_kernel<<<grid_for(g.n * x.Wh), kThreads, 0, st>>>(x);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace sc
