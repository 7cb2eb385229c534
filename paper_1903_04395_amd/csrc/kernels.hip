// gfx950 kernels for the colour-coding DP (Chen et al., HPDC'19).
//
//  * colouring            -- SplitMix64 counter-based colours (Section 2.1, phase 1)
//  * neighbour sum (SpMM) -- N = A * M_p over all passive columns at once
//                            (Eq. 2 and Section 4.2: one traversal per passive
//                            colour set; Section 4.5: SpMM)
//  * colour histogram     -- the same neighbour sum when the passive child is a
//                            single vertex (its table is the colour indicator)
//  * select / eMA         -- M_s[v,C] = sum_{C1 (+) C2 = C} M_a[v,C1] * N[v,C2]
//                            (Algorithm 4's element-wise multiply-add), with
//                            the a = 1 case reduced to a gather
//  * fused step           -- neighbour sum kept in LDS and consumed in place
//  * root reduction       -- colourful count per colouring
//
// All arithmetic is exact uint64 modulo 2^64; every carry out of 64 bits sets
// the colouring's bit in a 64-bit flag mask (bit r = colouring r of the pass).
#include "kernels.h"

namespace sc {
namespace kern {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t wave_or(uint64_t m) {
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, o, kWave);
        hi |= (uint32_t)__shfl_xor((int)hi, o, kWave);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Must be called by every lane of the wavefront (no lane may have exited).
__device__ __forceinline__ void flush_flags(uint64_t m, unsigned long long *flags) {
    if (__any(m != 0)) {
        uint64_t all = wave_or(m);
        if ((threadIdx.x & (kWave - 1)) == 0) atomicOr(flags, (unsigned long long)all);
    }
}

// acc + a*b with the exact-overflow rule: flag if a*b >= 2^64 or the sum carries.
__device__ __forceinline__ uint64_t mad_ovf(uint64_t acc, uint64_t a, uint64_t b, uint32_t &ovf) {
    uint64_t lo = a * b;
    uint64_t hi = __umul64hi(a, b);
    uint64_t s = acc + lo;
    ovf |= (uint32_t)(hi != 0) | (uint32_t)(s < lo);
    return s;
}

// ------------------------------------------------------------------ colours

__global__ __launch_bounds__(kBlock) void color_kernel(uint64_t seed, uint64_t first, int64_t n,
                                                      int B, int k, uint8_t *__restrict__ col) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n * B) return;
    int64_t v = i / B;
    int64_t r = i - v * B;
    uint64_t idx = ((first + (uint64_t)r) << 40) + (uint64_t)v;
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;     // SplitMix64 state
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;                // its finaliser
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    col[i] = (uint8_t)__umul64hi(z, (uint64_t)k);
}

// ------------------------------------------------------------------ neighbour sum

// One wavefront per light row and column chunk of 64*U uint64.
template <int U>
__global__ __launch_bounds__(kBlock) void spmm_light_kernel(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ rows, int64_t nrows, const uint64_t *__restrict__ P,
    uint64_t *__restrict__ N, int64_t L, int B, unsigned long long *__restrict__ flags) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t ri = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
    if (ri >= nrows) return;                                   // whole wavefront
    const int v = __builtin_amdgcn_readfirstlane(rows[ri]);
    const int64_t c0 = (int64_t)blockIdx.y * (kWave * U) + lane;
    const int64_t e0 = rp[v], e1 = rp[v + 1];
    uint64_t acc[U];
    bool inb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { acc[u] = 0; inb[u] = c0 + kWave * u < L; }
    uint32_t carry = 0;
    int64_t e = e0;
    for (; e + 2 <= e1; e += 2) {
        const uint64_t *s0 = P + (int64_t)ci[e] * L + c0;
        const uint64_t *s1 = P + (int64_t)ci[e + 1] * L + c0;
        uint64_t x0[U], x1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) { x0[u] = inb[u] ? s0[kWave * u] : 0; x1[u] = inb[u] ? s1[kWave * u] : 0; }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t s = acc[u] + x0[u];
            carry |= (uint32_t)(s < x0[u]) << u;
            uint64_t t = s + x1[u];
            carry |= (uint32_t)(t < x1[u]) << u;
            acc[u] = t;
        }
    }
    if (e < e1) {
        const uint64_t *s0 = P + (int64_t)ci[e] * L + c0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t x = inb[u] ? s0[kWave * u] : 0;
            uint64_t s = acc[u] + x;
            carry |= (uint32_t)(s < x) << u;
            acc[u] = s;
        }
    }
    uint64_t *d = N + (int64_t)v * L + c0;
    uint64_t m = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (inb[u]) d[kWave * u] = acc[u];
        if (carry & (1u << u)) m |= 1ull << ((c0 + kWave * u) % B);
    }
    flush_flags(m, flags);
}

// One workgroup (4 wavefronts splitting the neighbours) per wide item
// (row, segment) and column chunk.  Rows with more than `seg` neighbours are
// split; their segments add into N with atomics (N zeroed beforehand) and the
// returned old value exposes the carry.  `slot` (optional) redirects the output
// row: out_row = slot[v].
template <int U>
__global__ __launch_bounds__(kBlock) void spmm_wide_kernel(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int2 *__restrict__ items, int64_t nitems, int seg, const int32_t *__restrict__ slot,
    const uint64_t *__restrict__ P, uint64_t *__restrict__ N, int64_t L, int B,
    unsigned long long *__restrict__ flags) {
    __shared__ uint64_t red[kBlock / kWave - 1][U][kWave];
    __shared__ uint32_t redc[kBlock / kWave - 1][kWave];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int2 it = items[blockIdx.x];
    const int v = it.x;
    const int64_t r0 = rp[v], r1 = rp[v + 1];
    const int64_t e0 = r0 + (int64_t)it.y * seg;
    const int64_t e1 = min(e0 + seg, r1);
    const bool split = (r1 - r0) > seg;
    const int64_t c0 = (int64_t)blockIdx.y * (kWave * U) + lane;
    uint64_t acc[U];
    bool inb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { acc[u] = 0; inb[u] = c0 + kWave * u < L; }
    uint32_t carry = 0;
    for (int64_t e = e0 + wave; e < e1; e += kBlock / kWave) {
        const uint64_t *s0 = P + (int64_t)ci[e] * L + c0;
        uint64_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = inb[u] ? s0[kWave * u] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t s = acc[u] + x[u];
            carry |= (uint32_t)(s < x[u]) << u;
            acc[u] = s;
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) red[wave - 1][u][lane] = acc[u];
        redc[wave - 1][lane] = carry;
    }
    __syncthreads();
    uint64_t m = 0;
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < kBlock / kWave - 1; ++w) {
            carry |= redc[w][lane];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint64_t x = red[w][u][lane];
                uint64_t s = acc[u] + x;
                carry |= (uint32_t)(s < x) << u;
                acc[u] = s;
            }
        }
        const int64_t orow = slot ? (int64_t)slot[v] : (int64_t)v;
        uint64_t *d = N + orow * L + c0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!inb[u]) continue;
            if (split) {
                unsigned long long old = atomicAdd((unsigned long long *)(d + kWave * u),
                                                   (unsigned long long)acc[u]);
                if ((uint64_t)old + acc[u] < (uint64_t)old) carry |= 1u << u;
            } else {
                d[kWave * u] = acc[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (carry & (1u << u)) m |= 1ull << ((c0 + kWave * u) % B);
        flush_flags(m, flags);
    }
}

__global__ __launch_bounds__(kBlock) void zero_rows_kernel(const int32_t *__restrict__ rows,
                                                          int64_t nrows, const int32_t *slot,
                                                          uint64_t *__restrict__ N, int64_t L) {
    for (int64_t ri = blockIdx.y; ri < nrows; ri += gridDim.y) {
        const int v = rows[ri];
        const int64_t orow = slot ? (int64_t)slot[v] : (int64_t)v;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < L; c += (int64_t)gridDim.x * kBlock)
            N[orow * L + c] = 0;
    }
}

// ------------------------------------------------------------------ colour histogram (p = 1)

// One wavefront per light row; lanes are (neighbour slot, colouring) pairs;
// per-wavefront histograms of B*k uint32 counters live in LDS.
__global__ __launch_bounds__(kBlock) void hist_light_kernel(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ rows, int64_t nrows, const uint8_t *__restrict__ col,
    uint64_t *__restrict__ N, int B, int k) {
    extern __shared__ uint32_t hist_lds[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t *h = hist_lds + wave * B * k;
    const int64_t ri = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
    const bool valid = ri < nrows;
    for (int q = lane; q < B * k; q += kWave) h[q] = 0;
    __syncthreads();
    int v = 0;
    if (valid) {
        v = rows[ri];
        const int slots = kWave / B;
        const int s = lane / B, r = lane - (lane / B) * B;
        if (s < slots) {
            for (int64_t e = rp[v] + s; e < rp[v + 1]; e += slots) {
                const int c = col[(int64_t)ci[e] * B + r];
                atomicAdd(&h[r * k + c], 1u);
            }
        }
    }
    __syncthreads();
    if (valid) {
        uint64_t *d = N + (int64_t)v * k * B;
        for (int q = lane; q < B * k; q += kWave) {
            const int c = q / B, r = q - c * B;
            d[q] = h[r * k + c];
        }
    }
}

// One workgroup per wide item; rows split over several items add with atomics.
__global__ __launch_bounds__(kBlock) void hist_wide_kernel(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int2 *__restrict__ items, int64_t nitems, int seg, const int32_t *__restrict__ slot,
    const uint8_t *__restrict__ col, uint64_t *__restrict__ N, int B, int k) {
    extern __shared__ uint32_t hist_lds[];
    for (int q = threadIdx.x; q < B * k; q += kBlock) hist_lds[q] = 0;
    __syncthreads();
    const int2 it = items[blockIdx.x];
    const int v = it.x;
    const int64_t r0 = rp[v], r1 = rp[v + 1];
    const int64_t e0 = r0 + (int64_t)it.y * seg;
    const int64_t e1 = min(e0 + seg, r1);
    const bool split = (r1 - r0) > seg;
    const int slots = kBlock / B;
    const int s = threadIdx.x / B, r = threadIdx.x - s * B;
    if (s < slots)
        for (int64_t e = e0 + s; e < e1; e += slots) {
            const int c = col[(int64_t)ci[e] * B + r];
            atomicAdd(&hist_lds[r * k + c], 1u);
        }
    __syncthreads();
    const int64_t orow = slot ? (int64_t)slot[v] : (int64_t)v;
    uint64_t *d = N + orow * k * B;
    for (int q = threadIdx.x; q < B * k; q += kBlock) {
        const int c = q / B, rr = q - c * B;
        const uint64_t x = hist_lds[rr * k + c];
        if (split) {
            if (x) atomicAdd((unsigned long long *)(d + q), (unsigned long long)x);
        } else {
            d[q] = x;
        }
    }
}

// ------------------------------------------------------------------ select (a = 1) and eMA (a >= 2)

// grid: x over output columns of a row (Wh*B), y strides over rows.
__global__ __launch_bounds__(kBlock) void select_kernel(
    int64_t n, const uint8_t *__restrict__ col, const uint64_t *__restrict__ N,
    uint64_t *__restrict__ S, int B, int k, int Wh, int Wp, const int16_t *__restrict__ drop) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    const int Ls = Wh * B, Lp = Wp * B;
    if (q >= Ls) return;
    const int I = q / B, r = q - I * B;
    for (int64_t v = blockIdx.y; v < n; v += gridDim.y) {
        const int c = col[v * B + r];
        const int d = drop[I * k + c];
        S[v * Ls + q] = d >= 0 ? N[v * Lp + d * B + r] : 0;
    }
}

__global__ __launch_bounds__(kBlock) void ema_kernel(
    int64_t n, const uint64_t *__restrict__ A, const uint64_t *__restrict__ N,
    uint64_t *__restrict__ S, int B, int Wa, int Wp, int Wh, int nsplit,
    const uint32_t *__restrict__ split, unsigned long long *__restrict__ flags) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    const int Ls = Wh * B, La = Wa * B, Lp = Wp * B;
    const bool valid = q < Ls;
    const int I = valid ? q / B : 0, r = valid ? q - I * B : 0;
    uint64_t m = 0;
    for (int64_t v = blockIdx.y; v < n; v += gridDim.y) {
        if (valid) {
            const uint64_t *ra = A + v * La + r;
            const uint64_t *rn = N + v * Lp + r;
            const uint32_t *sp = split + (int64_t)I * nsplit;
            uint64_t acc = 0;
            uint32_t ovf = 0;
            for (int j = 0; j < nsplit; ++j) {
                const uint32_t pr = sp[j];
                acc = mad_ovf(acc, ra[(pr & 0xffff) * B], rn[(pr >> 16) * B], ovf);
            }
            S[v * Ls + q] = acc;
            if (ovf) m |= 1ull << r;
        }
    }
    flush_flags(m, flags);
}

// ------------------------------------------------------------------ fused step

// One workgroup per row.  Phase 1 builds the neighbour-sum row in LDS (colour
// histogram for p = 1, neighbour-row sum for p >= 2; rows whose neighbour sum
// was precomputed into `Npre` (slot[v] >= 0) copy it instead).  Phase 2 stages
// the active row (a >= 2).  Phase 3 writes the output row.
template <int U>
__global__ __launch_bounds__(kBlock) void fused_kernel(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ slot, const uint64_t *__restrict__ Npre,
    const uint8_t *__restrict__ col, const uint64_t *__restrict__ P,
    const uint64_t *__restrict__ A, uint64_t *__restrict__ S, int B, int k, int a, int p,
    int Wa, int Wp, int Wh, int nsplit, const uint32_t *__restrict__ split,
    const int16_t *__restrict__ drop, unsigned long long *__restrict__ flags) {
    extern __shared__ uint64_t lds[];
    const int64_t v = blockIdx.x;
    const int Lp = Wp * B, La = Wa * B, Ls = Wh * B;
    uint64_t *Nr = lds;                 // Lp words
    uint64_t *Ar = lds + Lp;            // La words (a >= 2)
    const int t = threadIdx.x;
    uint64_t m = 0;
    const int sv = slot ? slot[v] : -1;
    const int64_t e0 = rp[v], e1 = rp[v + 1];
    if (sv >= 0) {
        for (int q = t; q < Lp; q += kBlock) Nr[q] = Npre[(int64_t)sv * Lp + q];
    } else if (p == 1) {
        uint32_t *h = (uint32_t *)(lds + Lp + (a > 1 ? La : 0));   // k*B counters
        for (int q = t; q < Lp; q += kBlock) h[q] = 0;
        __syncthreads();
        const int slots = kBlock / B;
        const int s = t / B, r = t - s * B;
        if (s < slots)
            for (int64_t e = e0 + s; e < e1; e += slots)
                atomicAdd(&h[(int)col[(int64_t)ci[e] * B + r] * B + r], 1u);
        __syncthreads();
        for (int q = t; q < Lp; q += kBlock) Nr[q] = h[q];
    } else {
        uint64_t acc[U];
        uint32_t carry = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = 0;
        for (int64_t e = e0; e < e1; ++e) {
            const uint64_t *src = P + (int64_t)ci[e] * Lp + t;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (t + kBlock * u < Lp) {
                    const uint64_t x = src[kBlock * u];
                    const uint64_t s = acc[u] + x;
                    carry |= (uint32_t)(s < x) << u;
                    acc[u] = s;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = t + kBlock * u;
            if (q < Lp) {
                Nr[q] = acc[u];
                if (carry & (1u << u)) m |= 1ull << (q % B);
            }
        }
    }
    if (a > 1)
        for (int q = t; q < La; q += kBlock) Ar[q] = A[v * La + q];
    __syncthreads();
    uint64_t *out = S + v * Ls;
    if (a == 1) {
        for (int q = t; q < Ls; q += kBlock) {
            const int I = q / B, r = q - I * B;
            const int c = col[v * B + r];
            const int d = drop[I * k + c];
            out[q] = d >= 0 ? Nr[d * B + r] : 0;
        }
    } else {
        for (int q = t; q < Ls; q += kBlock) {
            const int I = q / B, r = q - I * B;
            const uint32_t *sp = split + (int64_t)I * nsplit;
            uint64_t acc = 0;
            uint32_t ovf = 0;
            for (int j = 0; j < nsplit; ++j) {
                const uint32_t pr = sp[j];
                acc = mad_ovf(acc, Ar[(pr & 0xffff) * B + r], Nr[(pr >> 16) * B + r], ovf);
            }
            out[q] = acc;
            if (ovf) m |= 1ull << r;
        }
    }
    flush_flags(m, flags);
}

// ------------------------------------------------------------------ root reduction

// grid: (blocks, B); block y = colouring r sums entries (v, I) of that colouring.
__global__ __launch_bounds__(kBlock) void reduce_kernel(int64_t n, const uint64_t *__restrict__ S,
                                                       int W, int B, unsigned long long *__restrict__ X,
                                                       unsigned long long *__restrict__ flags) {
    __shared__ uint64_t part[kBlock];
    __shared__ uint32_t cpart[kBlock];
    const int r = blockIdx.y;
    const int64_t total = n * W;
    uint64_t acc = 0;
    uint32_t carry = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const uint64_t x = S[i * B + r];
        const uint64_t s = acc + x;
        carry |= s < x;
        acc = s;
    }
    part[threadIdx.x] = acc;
    cpart[threadIdx.x] = carry;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const uint64_t x = part[threadIdx.x + w];
            const uint64_t s = part[threadIdx.x] + x;
            cpart[threadIdx.x] |= cpart[threadIdx.x + w] | (s < x);
            part[threadIdx.x] = s;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long old = atomicAdd(&X[r], (unsigned long long)part[0]);
        if (cpart[0] || (uint64_t)old + part[0] < (uint64_t)old) atomicOr(flags, 1ull << r);
    }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(uint64_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0;
}

inline unsigned row_grid(int64_t n) { return (unsigned)std::min<int64_t>(n, 65535); }

inline int pick_u(int64_t L) {
    // columns per lane for the neighbour-sum kernels: one chunk of 64*U per wavefront
    return L <= 64 ? 1 : (L <= 128 ? 2 : 4);
}

}  // namespace

hipError_t launch_zero_u64(uint64_t *p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = std::min<int64_t>((count + kBlock - 1) / kBlock, 8192);
    zero_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_color(uint64_t seed, uint64_t first, int64_t n, int B, int k, uint8_t *col,
                        hipStream_t st) {
    const int64_t total = n * B;
    if (total <= 0) return hipSuccess;
    color_kernel<<<dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(
        seed, first, n, B, k, col);
    return hipGetLastError();
}

template <int U>
static hipError_t spmm_u(const GraphBins &g, const uint64_t *P, uint64_t *N, int64_t L, int B,
                         unsigned long long *flags, hipStream_t st) {
    const unsigned chunks = (unsigned)((L + kWave * U - 1) / (kWave * U));
    if (g.n_split > 0) {
        zero_rows_kernel<<<dim3((unsigned)std::min<int64_t>((L + kBlock - 1) / kBlock, 64),
                                row_grid(g.n_split)), dim3(kBlock), 0, st>>>(
            g.split_rows, g.n_split, nullptr, N, L);
    }
    if (g.n_light > 0) {
        spmm_light_kernel<U><<<dim3((unsigned)((g.n_light + 3) / 4), chunks), dim3(kBlock), 0, st>>>(
            g.row_ptr, g.col_idx, g.light_rows, g.n_light, P, N, L, B, flags);
    }
    if (g.n_wide > 0) {
        spmm_wide_kernel<U><<<dim3((unsigned)g.n_wide, chunks), dim3(kBlock), 0, st>>>(
            g.row_ptr, g.col_idx, g.wide_items, g.n_wide, g.seg, nullptr, P, N, L, B, flags);
    }
    return hipGetLastError();
}

hipError_t launch_spmm(const GraphBins &g, const uint64_t *P, uint64_t *N, int64_t L, int B,
                       int chunk_cols, unsigned long long *flags, hipStream_t st) {
    int u = chunk_cols > 0 ? std::max(1, std::min(4, chunk_cols / kWave)) : pick_u(L);
    if (u >= 4) return spmm_u<4>(g, P, N, L, B, flags, st);
    if (u >= 2) return spmm_u<2>(g, P, N, L, B, flags, st);
    return spmm_u<1>(g, P, N, L, B, flags, st);
}

hipError_t launch_hist(const GraphBins &g, const uint8_t *col, uint64_t *N, int B, int k,
                       hipStream_t st) {
    const int64_t L = (int64_t)k * B;
    if (g.n_split > 0) {
        zero_rows_kernel<<<dim3(1, row_grid(g.n_split)), dim3(kBlock), 0, st>>>(
            g.split_rows, g.n_split, nullptr, N, L);
    }
    if (g.n_light > 0) {
        hist_light_kernel<<<dim3((unsigned)((g.n_light + 3) / 4)), dim3(kBlock),
                            (size_t)4 * B * k * sizeof(uint32_t), st>>>(
            g.row_ptr, g.col_idx, g.light_rows, g.n_light, col, N, B, k);
    }
    if (g.n_wide > 0) {
        hist_wide_kernel<<<dim3((unsigned)g.n_wide), dim3(kBlock), (size_t)B * k * sizeof(uint32_t), st>>>(
            g.row_ptr, g.col_idx, g.wide_items, g.n_wide, g.seg, nullptr, col, N, B, k);
    }
    return hipGetLastError();
}

hipError_t launch_select(int64_t n, const uint8_t *col, const uint64_t *N, uint64_t *S, int B,
                         int k, int Wh, int Wp, const int16_t *drop, hipStream_t st) {
    const int Ls = Wh * B;
    if (n <= 0 || Ls <= 0) return hipSuccess;
    select_kernel<<<dim3((unsigned)((Ls + kBlock - 1) / kBlock), row_grid(n)), dim3(kBlock), 0, st>>>(
        n, col, N, S, B, k, Wh, Wp, drop);
    return hipGetLastError();
}

hipError_t launch_ema(int64_t n, const uint64_t *A, const uint64_t *N, uint64_t *S, int B,
                      int Wa, int Wp, int Wh, int nsplit, const uint32_t *split,
                      unsigned long long *flags, hipStream_t st) {
    const int Ls = Wh * B;
    if (n <= 0 || Ls <= 0) return hipSuccess;
    ema_kernel<<<dim3((unsigned)((Ls + kBlock - 1) / kBlock), row_grid(n)), dim3(kBlock), 0, st>>>(
        n, A, N, S, B, Wa, Wp, Wh, nsplit, split, flags);
    return hipGetLastError();
}

template <int U>
static void fused_u(const GraphBins &g, const int32_t *slot, const uint64_t *Npre,
                    const uint8_t *col, const uint64_t *P, const uint64_t *A, uint64_t *S, int B,
                    int k, int a, int p, int Wa, int Wp, int Wh, int nsplit,
                    const uint32_t *split, const int16_t *drop, unsigned long long *flags,
                    size_t lds, hipStream_t st) {
    fused_kernel<U><<<dim3((unsigned)g.n), dim3(kBlock), lds, st>>>(
        g.row_ptr, g.col_idx, slot, Npre, col, P, A, S, B, k, a, p, Wa, Wp, Wh, nsplit, split,
        drop, flags);
}

hipError_t launch_fused(const GraphBins &g, const uint8_t *col, const uint64_t *P,
                        const uint64_t *A, uint64_t *S, int B, int k, int a, int p, int Wa,
                        int Wp, int Wh, int nsplit, const uint32_t *split, const int16_t *drop,
                        unsigned long long *flags, hipStream_t st) {
    (void)g; (void)col; (void)P; (void)A; (void)S; (void)B; (void)k; (void)a; (void)p;
    (void)Wa; (void)Wp; (void)Wh; (void)nsplit; (void)split; (void)drop; (void)flags; (void)st;
    return hipErrorNotSupported;
}

hipError_t launch_reduce(int64_t n, const uint64_t *S, int W, int B, unsigned long long *X,
                         unsigned long long *flags, hipStream_t st) {
    if (n <= 0 || B <= 0) return hipSuccess;
    const int64_t total = n * W;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kBlock - 1) / kBlock, 1024));
    reduce_kernel<<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, B, X, flags);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace sc
