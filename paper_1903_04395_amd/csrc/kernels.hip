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
// A launch may hold at most 2^32 - 1 work-items per grid dimension; kernels
// that stride over their items are launched with at most this many workgroups.
constexpr int64_t kMaxStrideBlocks = 1 << 16;
constexpr int64_t kMaxGridBlocks = ((int64_t)1 << 32) / kBlock - 1;

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

// col[v*B + r]: colour of internal vertex v (original id perm[v], or v) in
// colouring first + r, with desc = {seed, first} read from device memory so a
// captured pass can be replayed for any colouring range.
__global__ __launch_bounds__(kBlock) void color_kernel(const uint64_t *__restrict__ desc, int64_t n,
                                                      int B, int k, const int32_t *__restrict__ perm,
                                                      uint8_t *__restrict__ col) {
    const uint64_t seed = desc[0], first = desc[1];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n * B;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t v = i / B;
        const int64_t r = i - v * B;
        const uint64_t orig = perm ? (uint64_t)perm[v] : (uint64_t)v;
        const uint64_t idx = ((first + (uint64_t)r) << 40) + orig;
        uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;     // SplitMix64 state
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;                // its finaliser
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        col[i] = (uint8_t)__umul64hi(z, (uint64_t)k);
    }
}

// ------------------------------------------------------------------ neighbour sum

// Accumulates P rows of the neighbours e0, e0+step, ... < e1 into acc[] for
// the lane's U columns c0 + 64u (bounds in inb[]), four neighbours at a time
// so that 4*U loads are in flight per lane.
template <int U>
__device__ __forceinline__ void gather_rows(int64_t e0, int64_t e1, int step,
                                            const int32_t *__restrict__ ci,
                                            const uint64_t *__restrict__ P, int64_t L, int64_t c0,
                                            const bool (&inb)[U], uint64_t (&acc)[U],
                                            uint32_t &carry) {
    int64_t e = e0;
    for (; e + 3 * step < e1; e += 4 * step) {
        const uint64_t *s[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = P + (int64_t)ci[e + i * step] * L + c0;
        uint64_t x[4][U];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u) x[i][u] = inb[u] ? s[i][kWave * u] : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t t = acc[u] + x[i][u];
                carry |= (uint32_t)(t < x[i][u]) << u;
                acc[u] = t;
            }
    }
    for (; e < e1; e += step) {
        const uint64_t *s0 = P + (int64_t)ci[e] * L + c0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t x = inb[u] ? s0[kWave * u] : 0;
            const uint64_t t = acc[u] + x;
            carry |= (uint32_t)(t < x) << u;
            acc[u] = t;
        }
    }
}

struct SpmmArgs {
    const int64_t *rp;
    const int32_t *ci;
    const int32_t *light;  int64_t n_light;   // light rows, 4 per workgroup
    const int2 *wide;      int64_t n_wide;    // (row, segment) items, 1 per workgroup
    int seg;
    const int32_t *slot;                      // optional output-row redirect
    const uint64_t *P;
    uint64_t *N;
    int64_t L;
    int B;
    int64_t groups;                           // light groups + wide items
    int64_t chunks;                           // column chunks of 64*U
    unsigned long long *flags;
};

// Neighbour sum N = A * P, tiled by column chunks of 64*U uint64 (a 2 KB
// contiguous slice of every gathered row for U = 4) and walked chunk-major so
// that the rows in flight read one chunk.  Light rows: one wavefront each,
// four per workgroup.  Wide items: four wavefronts split the neighbours and
// meet in LDS; rows with more than `seg` neighbours are split over several
// items whose partial sums meet in global atomics (the carry is read from the
// returned old value).  The grid strides over (chunk, group) items.
template <int U>
__device__ __forceinline__ void spmm_tiled_item(const SpmmArgs &a, int64_t chunk, int64_t g,
                                                uint64_t (*red)[U][kWave], uint32_t (*redc)[kWave]) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c0 = chunk * (kWave * U) + lane;
    bool inb[U];
    uint64_t acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { inb[u] = c0 + kWave * u < a.L; acc[u] = 0; }
    uint32_t carry = 0;
    const int64_t nlg = (a.n_light + 3) >> 2;
    if (g < nlg) {
        const int64_t li = g * 4 + wave;
        if (li >= a.n_light) return;                   // whole wavefront, this item only
        const int v = __builtin_amdgcn_readfirstlane(a.light[li]);
        gather_rows<U>(a.rp[v], a.rp[v + 1], 1, a.ci, a.P, a.L, c0, inb, acc, carry);
        uint64_t *d = a.N + (int64_t)v * a.L + c0;
        uint64_t m = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (inb[u]) d[kWave * u] = acc[u];
            if (carry & (1u << u)) m |= 1ull << ((c0 + kWave * u) % a.B);
        }
        flush_flags(m, a.flags);
        return;
    }
    const int2 it = a.wide[g - nlg];
    const int v = __builtin_amdgcn_readfirstlane(it.x);
    const int64_t r0 = a.rp[v], r1 = a.rp[v + 1];
    const int64_t e0 = r0 + (int64_t)it.y * a.seg;
    const int64_t e1 = min(e0 + a.seg, r1);
    const bool split = (r1 - r0) > a.seg;
    gather_rows<U>(e0 + wave, e1, kBlock / kWave, a.ci, a.P, a.L, c0, inb, acc, carry);
    if (wave > 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) red[wave - 1][u][lane] = acc[u];
        redc[wave - 1][lane] = carry;
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < kBlock / kWave - 1; ++w) {
            carry |= redc[w][lane];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t x = red[w][u][lane];
                const uint64_t t = acc[u] + x;
                carry |= (uint32_t)(t < x) << u;
                acc[u] = t;
            }
        }
        const int64_t orow = a.slot ? (int64_t)a.slot[v] : (int64_t)v;
        uint64_t *d = a.N + orow * a.L + c0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!inb[u]) continue;
            if (split) {
                const unsigned long long old = atomicAdd((unsigned long long *)(d + kWave * u),
                                                         (unsigned long long)acc[u]);
                if ((uint64_t)old + acc[u] < (uint64_t)old) carry |= 1u << u;
            } else {
                d[kWave * u] = acc[u];
            }
        }
        uint64_t m = 0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (carry & (1u << u)) m |= 1ull << ((c0 + kWave * u) % a.B);
        flush_flags(m, a.flags);
    }
}

// PRE (a distinct instantiation, so profiles tell the two apart): the pre-pass
// that sums only the split rows into the compact buffer.
template <int U, bool PRE>
__global__ __launch_bounds__(kBlock) void spmm_tiled_kernel(SpmmArgs a) {
    __shared__ uint64_t red[kBlock / kWave - 1][U][kWave];
    __shared__ uint32_t redc[kBlock / kWave - 1][kWave];
    const int64_t total = a.chunks * a.groups;
    const int64_t nlg = (a.n_light + 3) >> 2;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t chunk = b / a.groups, g = b - chunk * a.groups;
        spmm_tiled_item<U>(a, chunk, g, red, redc);
        if (g >= nlg) __syncthreads();                 // red/redc reused by the next wide item
    }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int mask) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, mask, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), mask, kWave);
    return ((uint64_t)hi << 32) | lo;
}

struct NarrowArgs {
    const int64_t *rp;
    const int32_t *ci;
    const int2 *tasks;        // (row, segment of `seg` neighbours)
    int64_t n_tasks;
    int seg;
    const int32_t *slot;      // optional output-row redirect
    const uint64_t *P;
    uint64_t *N;
    int64_t L;
    int B;
    int64_t tiles;            // column tiles of Z uint64
    unsigned long long *flags;
};

// Neighbour sum N = A * P in narrow column tiles of Z uint64 (Z*8 bytes of
// every gathered row per tile).  The tiles are walked one after another over
// all rows, so while a tile is in flight only n*Z*8 bytes of P are live: the
// hub rows' tile slices stay in L2 and the whole tile fits the last-level
// cache.  One wavefront per (tile, task): its 64 lanes are 64/Z groups of Z
// lanes; each group walks every (64/Z)-th neighbour of the task (four in
// flight) and the groups are summed with cross-lane shuffles.  A task is a
// whole row, or a `seg`-neighbour segment of a row with more neighbours,
// whose partial sums meet in global atomics (N zeroed beforehand; the carry is
// read from the returned old value).
template <int Z>
__global__ __launch_bounds__(kBlock) void spmm_narrow_kernel(NarrowArgs a) {
    constexpr int G = kWave / Z;
    const int lane = threadIdx.x & (kWave - 1);
    const int grp = lane / Z, cz = lane - (lane / Z) * Z;
    const int64_t total = a.tiles * a.n_tasks;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / kWave);
    // items in (tile, task) order; the grid strides over them, so the items in
    // flight at any time belong to one or two consecutive tiles
    for (int64_t wid = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6); wid < total;
         wid += stride) {
        const int64_t tile = wid / a.n_tasks;
        const int64_t ti = wid - tile * a.n_tasks;
        const int2 tk = a.tasks[ti];
        const int v = tk.x;
        const int64_t r0 = a.rp[v], r1 = a.rp[v + 1];
        const int64_t e0 = r0 + (int64_t)tk.y * a.seg;
        const int64_t e1 = min(e0 + a.seg, r1);
        const bool split = (r1 - r0) > a.seg;
        const int64_t c = tile * Z + cz;
        const bool inb = c < a.L;
        const uint64_t *Pc = a.P + c;
        uint64_t acc = 0;
        uint32_t carry = 0;
        int64_t e = e0 + grp;
        for (; e + 3 * G < e1; e += 4 * G) {
            const int64_t j0 = a.ci[e], j1 = a.ci[e + G], j2 = a.ci[e + 2 * G], j3 = a.ci[e + 3 * G];
            const uint64_t x0 = inb ? Pc[j0 * a.L] : 0, x1 = inb ? Pc[j1 * a.L] : 0;
            const uint64_t x2 = inb ? Pc[j2 * a.L] : 0, x3 = inb ? Pc[j3 * a.L] : 0;
            uint64_t t = acc + x0; carry |= t < x0;
            acc = t + x1;          carry |= acc < x1;
            t = acc + x2;          carry |= t < x2;
            acc = t + x3;          carry |= acc < x3;
        }
        for (; e < e1; e += G) {
            const uint64_t x = inb ? Pc[(int64_t)a.ci[e] * a.L] : 0;
            const uint64_t t = acc + x;
            carry |= t < x;
            acc = t;
        }
#pragma unroll
        for (int o = Z; o < kWave; o <<= 1) {
            const uint64_t y = shfl_xor_u64(acc, o);
            carry |= (uint32_t)__shfl_xor((int)carry, o, kWave);
            const uint64_t t = acc + y;
            carry |= t < y;
            acc = t;
        }
        uint64_t m = 0;
        if (grp == 0 && inb) {
            const int64_t orow = a.slot ? (int64_t)a.slot[v] : (int64_t)v;
            uint64_t *d = a.N + orow * a.L + c;
            if (split) {
                const unsigned long long old = atomicAdd((unsigned long long *)d, (unsigned long long)acc);
                if ((uint64_t)old + acc < (uint64_t)old) carry = 1;
            } else {
                *d = acc;
            }
            if (carry) m = 1ull << (c % a.B);
        }
        flush_flags(m, a.flags);
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

// ------------------------------------------------------------------ row kernel

enum RowMode { kRowStaged = 0, kRowGather = 1, kRowHist = 2 };

struct RowArgs {
    const int64_t *rp;
    const int32_t *ci;
    const int32_t *slot;          // split rows: index into Npre, else -1 (may be NULL)
    const uint64_t *Npre;         // precomputed neighbour sums of split rows
    const uint8_t *col;
    const uint64_t *src;          // kRowStaged: N;  kRowGather: passive table P
    const uint64_t *A;            // active table (a >= 2)
    uint64_t *S;
    int B, k, a, Wa, Wp, Wh, nsplit;
    const uint32_t *split;
    const int16_t *drop;
    unsigned long long *flags;
    int64_t n;                    // rows
};

// One workgroup per graph row v (the grid strides over the rows).  The
// neighbour-sum row N[v] (Wp*B words) is built in LDS -- copied from N
// (staged), summed from the neighbours' passive
// rows (fused neighbour sum), or counted from the neighbours' colours (fused
// histogram, p = 1); split rows copy their precomputed sum.  The active row is
// staged next to it (a >= 2).  Every output entry (I, r) of S[v] is then
// either a select through the drop-colour table (a = 1) or the split sum
// sum_j A[v][Ia_j][r] * N[v][Ip_j][r] (a >= 2), read from LDS.
template <int MODE, int U>
__device__ __forceinline__ void row_body(const RowArgs &a, int64_t v, uint64_t *lds) {
    const int B = a.B;
    const int Lp = a.Wp * B, La = a.Wa * B, Ls = a.Wh * B;
    uint64_t *Nr = lds;
    uint64_t *Ar = lds + Lp;
    const int t = threadIdx.x;
    uint64_t m = 0;
    if (MODE == kRowStaged) {
        for (int q = t; q < Lp; q += kBlock) Nr[q] = a.src[v * Lp + q];
    } else {
        const int sv = a.slot ? a.slot[v] : -1;
        if (sv >= 0) {
            for (int q = t; q < Lp; q += kBlock) Nr[q] = a.Npre[(int64_t)sv * Lp + q];
        } else if (MODE == kRowHist) {
            uint32_t *h = (uint32_t *)(lds + Lp + (a.a > 1 ? La : 0));
            for (int q = t; q < Lp; q += kBlock) h[q] = 0;
            __syncthreads();
            const int slots = kBlock / B;
            const int s = t / B, r = t - s * B;
            if (s < slots)
                for (int64_t e = a.rp[v] + s; e < a.rp[v + 1]; e += slots)
                    atomicAdd(&h[(int)a.col[(int64_t)a.ci[e] * B + r] * B + r], 1u);
            __syncthreads();
            for (int q = t; q < Lp; q += kBlock) Nr[q] = h[q];
        } else {
            // fused neighbour sum: wavefront w owns columns [w*64U, (w+1)*64U)
            bool inb[U];
            uint64_t acc[U];
            const int lane = t & (kWave - 1);
            const int64_t cw = (int64_t)(t >> 6) * kWave * U + lane;   // wave-contiguous columns
#pragma unroll
            for (int u = 0; u < U; ++u) { inb[u] = cw + kWave * u < Lp; acc[u] = 0; }
            uint32_t carry = 0;
            gather_rows<U>(a.rp[v], a.rp[v + 1], 1, a.ci, a.src, Lp, cw, inb, acc, carry);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (inb[u]) Nr[cw + kWave * u] = acc[u];
                if (carry & (1u << u)) m |= 1ull << ((cw + kWave * u) % B);
            }
        }
    }
    if (a.a > 1)
        for (int q = t; q < La; q += kBlock) Ar[q] = a.A[v * La + q];
    __syncthreads();
    uint64_t *out = a.S + v * Ls;
    if (a.a == 1) {
        const uint8_t *cv = a.col + v * B;
        for (int q = t; q < Ls; q += kBlock) {
            const int I = q / B, r = q - I * B;
            const int d = a.drop[I * a.k + cv[r]];
            out[q] = d >= 0 ? Nr[d * B + r] : 0;
        }
    } else {
        for (int q = t; q < Ls; q += kBlock) {
            const int I = q / B, r = q - I * B;
            const uint32_t *sp = a.split + (int64_t)I * a.nsplit;
            uint64_t acc = 0;
            uint32_t ovf = 0;
            for (int j = 0; j < a.nsplit; ++j) {
                const uint32_t pr = sp[j];
                acc = mad_ovf(acc, Ar[(pr & 0xffff) * B + r], Nr[(pr >> 16) * B + r], ovf);
            }
            out[q] = acc;
            if (ovf) m |= 1ull << r;
        }
    }
    flush_flags(m, a.flags);
}

template <int MODE, int U>
__global__ __launch_bounds__(kBlock) void row_kernel(RowArgs a) {
    extern __shared__ uint64_t lds[];
    for (int64_t v = blockIdx.x; v < a.n; v += gridDim.x) {
        row_body<MODE, U>(a, v, lds);
        __syncthreads();                      // LDS is reused by the next row
    }
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

hipError_t launch_color(const uint64_t *desc, int64_t n, int B, int k, const int32_t *perm,
                        uint8_t *col, hipStream_t st) {
    const int64_t total = n * B;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, kMaxStrideBlocks);
    color_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(desc, n, B, k, perm, col);
    return hipGetLastError();
}

template <int U>
static hipError_t spmm_tiled_u(const GraphBins &g, bool split_only, const uint64_t *P, uint64_t *N,
                               int64_t L, int B, unsigned long long *flags, hipStream_t st) {
    const int32_t *slot = split_only ? g.slot : nullptr;
    SpmmArgs a;
    a.rp = g.row_ptr; a.ci = g.col_idx;
    a.light = g.light_rows; a.n_light = split_only ? 0 : g.n_light;
    a.wide = g.wide_items; a.n_wide = split_only ? g.n_split_items : g.n_wide;
    a.seg = g.seg; a.slot = slot; a.P = P; a.N = N; a.L = L; a.B = B;
    a.groups = ((a.n_light + 3) >> 2) + a.n_wide;
    a.chunks = (L + kWave * U - 1) / (kWave * U);
    a.flags = flags;
    if (a.groups == 0 || L <= 0) return hipGetLastError();
    // one workgroup per item while the grid allows it (the dispatcher then
    // balances uneven items); beyond that the workgroups stride
    const int64_t blocks = std::min<int64_t>(a.chunks * a.groups, kMaxGridBlocks);
    if (split_only) spmm_tiled_kernel<U, true><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(a);
    else spmm_tiled_kernel<U, false><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(a);
    return hipGetLastError();
}

template <int Z>
static hipError_t spmm_narrow_z(const GraphBins &g, bool split_only, const uint64_t *P,
                                uint64_t *N, int64_t L, int B, unsigned long long *flags,
                                hipStream_t st) {
    const int32_t *slot = split_only ? g.slot : nullptr;
    NarrowArgs a;
    a.rp = g.row_ptr; a.ci = g.col_idx;
    a.tasks = g.tasks; a.n_tasks = split_only ? g.n_split_tasks : g.n_tasks;
    a.seg = g.seg; a.slot = slot; a.P = P; a.N = N; a.L = L; a.B = B;
    a.tiles = (L + Z - 1) / Z;
    a.flags = flags;
    if (a.n_tasks == 0 || L <= 0) return hipGetLastError();
    const int64_t waves = a.tiles * a.n_tasks;
    const int64_t blocks = std::min<int64_t>((waves + kBlock / kWave - 1) / (kBlock / kWave), kMaxGridBlocks);
    spmm_narrow_kernel<Z><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(a);
    return hipGetLastError();
}

static hipError_t spmm_any(int tile_cols, const GraphBins &g, bool split_only, const uint64_t *P,
                           uint64_t *N, int64_t L, int B, unsigned long long *flags, hipStream_t st) {
    switch (tile_cols) {
    case 8: return spmm_narrow_z<8>(g, split_only, P, N, L, B, flags, st);
    case 16: return spmm_narrow_z<16>(g, split_only, P, N, L, B, flags, st);
    case 32: return spmm_narrow_z<32>(g, split_only, P, N, L, B, flags, st);
    case 64: return spmm_tiled_u<1>(g, split_only, P, N, L, B, flags, st);
    case 128: return spmm_tiled_u<2>(g, split_only, P, N, L, B, flags, st);
    default: return spmm_tiled_u<4>(g, split_only, P, N, L, B, flags, st);
    }
}

hipError_t launch_zero_split_rows(const GraphBins &g, bool compact, uint64_t *N, int64_t L,
                                  hipStream_t st) {
    if (g.n_split == 0 || L <= 0) return hipSuccess;
    zero_rows_kernel<<<dim3((unsigned)std::min<int64_t>((L + kBlock - 1) / kBlock, 64),
                            row_grid(g.n_split)), dim3(kBlock), 0, st>>>(
        g.split_rows, g.n_split, compact ? g.slot : nullptr, N, L);
    return hipGetLastError();
}

hipError_t launch_spmm(const GraphBins &g, const uint64_t *P, uint64_t *N, int64_t L, int B,
                       int tile_cols, unsigned long long *flags, hipStream_t st) {
    return spmm_any(tile_cols, g, false, P, N, L, B, flags, st);
}

hipError_t launch_spmm_split(const GraphBins &g, const uint64_t *P, uint64_t *Npre, int64_t L,
                             int B, int tile_cols, unsigned long long *flags, hipStream_t st) {
    if (g.n_split == 0) return hipSuccess;
    return spmm_any(tile_cols, g, true, P, Npre, L, B, flags, st);
}

hipError_t launch_hist_split(const GraphBins &g, const uint8_t *col, uint64_t *Npre, int B, int k,
                             hipStream_t st) {
    if (g.n_split == 0) return hipSuccess;
    const int64_t L = (int64_t)k * B;
    if (g.n_split_items > kMaxGridBlocks) return hipErrorInvalidValue;
    zero_rows_kernel<<<dim3(1, row_grid(g.n_split)), dim3(kBlock), 0, st>>>(
        g.split_rows, g.n_split, g.slot, Npre, L);
    hist_wide_kernel<<<dim3((unsigned)g.n_split_items), dim3(kBlock), (size_t)B * k * sizeof(uint32_t), st>>>(
        g.row_ptr, g.col_idx, g.wide_items, g.n_split_items, g.seg, g.slot, col, Npre, B, k);
    return hipGetLastError();
}

hipError_t launch_hist(const GraphBins &g, const uint8_t *col, uint64_t *N, int B, int k,
                       hipStream_t st) {
    const int64_t L = (int64_t)k * B;
    if (g.n_split > 0) {
        zero_rows_kernel<<<dim3(1, row_grid(g.n_split)), dim3(kBlock), 0, st>>>(
            g.split_rows, g.n_split, nullptr, N, L);
    }
    if ((g.n_light + 3) / 4 > kMaxGridBlocks || g.n_wide > kMaxGridBlocks) return hipErrorInvalidValue;
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

int row_lds_bytes(int k, int a, int Wa, int Wp, int B, int mode) {
    int64_t words = (int64_t)Wp * B + (a > 1 ? (int64_t)Wa * B : 0);
    int64_t bytes = words * 8 + (mode == kRowHist ? (int64_t)k * B * 4 : 0);
    return (int)bytes;
}

int row_max_u() { return 8; }

template <int MODE, int U>
static void row_u(const RowArgs &a, int64_t n, size_t lds, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>(n, kMaxGridBlocks);
    row_kernel<MODE, U><<<dim3((unsigned)blocks), dim3(kBlock), lds, st>>>(a);
}

hipError_t launch_row(int mode, const GraphBins &g, const uint8_t *col, const uint64_t *src,
                      const uint64_t *Npre, const uint64_t *A, uint64_t *S, int B, int k, int a,
                      int Wa, int Wp, int Wh, int nsplit, const uint32_t *split,
                      const int16_t *drop, unsigned long long *flags, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    RowArgs r;
    r.rp = g.row_ptr; r.ci = g.col_idx;
    r.slot = mode == kRowStaged ? nullptr : g.slot;
    r.Npre = Npre; r.col = col; r.src = src; r.A = A; r.S = S;
    r.B = B; r.k = k; r.a = a; r.Wa = Wa; r.Wp = Wp; r.Wh = Wh; r.nsplit = nsplit;
    r.split = split; r.drop = drop; r.flags = flags; r.n = g.n;
    const size_t lds = (size_t)row_lds_bytes(k, a, Wa, Wp, B, mode);
    const int64_t Lp = (int64_t)Wp * B;
    if (mode == kRowStaged) row_u<kRowStaged, 1>(r, g.n, lds, st);
    else if (mode == kRowHist) row_u<kRowHist, 1>(r, g.n, lds, st);
    else if (Lp <= 256) row_u<kRowGather, 1>(r, g.n, lds, st);
    else if (Lp <= 512) row_u<kRowGather, 2>(r, g.n, lds, st);
    else if (Lp <= 1024) row_u<kRowGather, 4>(r, g.n, lds, st);
    else if (Lp <= 2048) row_u<kRowGather, 8>(r, g.n, lds, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
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
