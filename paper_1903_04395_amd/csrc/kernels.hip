// gfx950 kernels for the colour-coding DP (Chen et al., HPDC'19).
//
//  * colouring    -- SplitMix64 counter-based colours (Section 2.1, phase 1)
//  * DP step      -- one row kernel per attach of a passive child: the
//                    neighbour sum N = A * M_p taken once per passive colour
//                    set (Eq. 2 with the pruning of Section 4.2; the SpMM of
//                    Section 4.5) built per row in LDS, then the element-wise
//                    multiply-add M_s[v,C] = sum_{C1 (+) C2 = C} M_a[v,C1] *
//                    N[v,C2] (Algorithm 4), fused, in the rooted-colour layout
//                    described in kernels.h
//  * split pre-pass -- the neighbour sums of rows with very many neighbours
//  * root reduction -- colourful count per colouring
//  * homomorphism bound -- the same steps on one double per vertex (an upper
//                    bound on every colouring's count)
//
// All arithmetic is exact uint64 modulo 2^64; every carry out of 64 bits sets
// the colouring's bit in a 64-bit flag mask (bit r = colouring r of the pass).
// In residue mode (MOD) the same kernels keep every entry modulo a prime
// instead, which with the uint64 pass recovers counts past 2^64.
//
// In the rooted-colour layout a neighbour u of v contributes its entry for the
// set {col(u)} + T (T a subset of the colours other than col(u)) to v's
// neighbour-sum entry for the same set, when that set does not hold col(v);
// the entry index is found by re-ranking the set among the colours other than
// col(v).  Sets that hold col(v) only ever meet zero active entries and are
// skipped, and neighbours that share v's colour contribute nothing.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "kernels.h"
#include "exact.h"      // after the HIP runtime header (it uses __device__)

namespace sc {
namespace kern {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// Steps whose rows need more than kWideLds bytes of LDS fit at most three
// workgroups per CU; they run 512-thread workgroups, so that twice as many
// wavefronts share each row's LDS.
constexpr int kBlockWide = 512;
constexpr int kWideLds = 48 * 1024;
// A launch may hold at most 2^32 - 1 work-items per grid dimension; kernels
// that stride over their items are launched with at most this many workgroups.
constexpr int64_t kMaxStrideBlocks = 1 << 16;
constexpr int kCUs = 256;
constexpr int kMaxBlocksPerCU = 8;    // 32 wavefronts of 4-wave workgroups
constexpr int kLdsPerCU = 160 * 1024;
constexpr int kSplitLdsMax = 4096;    // split-table entries staged in LDS (16 KB)
constexpr int kGroupRows = 3;         // chunk-count tag of the lane-group scatter
// (plane, row) items a step needs before it builds rows one per wavefront:
// four per wavefront slot of the chip
constexpr int64_t kWaveRowsMin = (int64_t)kCUs * kMaxBlocksPerCU * kWaves * 4;
constexpr int kMad3Pairs = 32;        // split pairs per entry from which the three-multiply
                                      // product is used (vector-ALU-bound multiply-adds)

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

// ------------------------------------------------------------------ DP step

struct DpArgs {
    const int64_t *rp;
    const int32_t *ci;
    const uint8_t *col;
    int64_t n;                    // table rows
    int B, Bi, sh, planes;        // sh = log2(Bi)
    int p, Wq, Wn, Wa, Wh, nsplit;
    int eg, lg_eg;                // lanes per output entry in the multiply-add (power of two)
    int split_lds;                // the split table is staged in LDS after the other tables
    const uint32_t *split;
    const uint16_t *unrank, *rank;
    int n_rank, rank_direct;      // rank_direct: `rank` holds every mask (2^(k-1) entries)
    const uint64_t *P, *A;
    uint64_t *S;
    uint64_t *Npre;
    const int32_t *slot;
    int64_t n_split;
    const int2 *items;            // split pre-pass: (row, segment)
    int64_t n_items;
    int seg;
    int tab_off;                  // LDS byte offset of the index tables
    Modulus md;                   // residue mode: the prime, its fold constants, 2^64 mod p
    unsigned long long *flags;
};

// The threads that build one row: the whole workgroup (four wavefronts, the
// row's neighbours split over them), or one wavefront on its own row.
struct Team {
    int wave, waves;      // this thread's wavefront within the team, wavefronts in the team
    int tid, size;        // this thread within the team, threads in the team
};

template <int TPB>
__device__ __forceinline__ Team block_team() {
    return Team{(int)(threadIdx.x >> 6), TPB / kWave, (int)threadIdx.x, TPB};
}

__device__ __forceinline__ Team wave_team() {
    return Team{0, 1, (int)(threadIdx.x & (kWave - 1)), kWave};
}

// Orders the team's LDS accesses: a workgroup barrier, or for a single
// wavefront (whose LDS operations complete in issue order) a fence that keeps
// the compiler from moving LDS accesses across it.
template <bool WAVE>
__device__ __forceinline__ void team_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Residue mode: a 64-bit word accumulates a value known only modulo p, so an
// add that wraps past 2^64 loses 2^64, which is put back as 2^64 mod p (an add
// that wraps again puts back once more).
__device__ __forceinline__ void put_back_wrap(unsigned long long *ptr, uint64_t wrap) {
    for (;;) {
        const unsigned long long o = atomicAdd(ptr, (unsigned long long)wrap);
        if ((uint64_t)o + wrap >= wrap) break;
    }
}

// Inserts a zero bit at position c (renumbered colours -> colours).
__device__ __forceinline__ uint32_t widen_at(uint32_t m, int c) {
    const uint32_t lo = m & ((1u << c) - 1u);
    return lo | ((m ^ lo) << 1);
}
// Removes bit c, which must be zero (colours -> colours other than c, renumbered).
__device__ __forceinline__ uint32_t narrow_at(uint32_t m, int c) {
    const uint32_t lo = m & ((1u << c) - 1u);
    return lo | ((m ^ lo) >> 1);
}

// Copies the index tables a step needs into LDS (called by the whole block):
// unrank and rank tables (p >= 2), then the split table when it fits.
template <int TPB>
__device__ __forceinline__ void stage_tables(const DpArgs &a, uint16_t *tab) {
    const int nt = a.p >= 2 ? a.Wq + a.n_rank : 0;
    if (a.p >= 2) {
        for (int i = threadIdx.x; i < a.Wq; i += TPB) tab[i] = a.unrank[i];
        for (int i = threadIdx.x; i < a.n_rank; i += TPB) tab[a.Wq + i] = a.rank[i];
    }
    if (a.split_lds) {
        uint32_t *sp = (uint32_t *)(tab + ((nt + 1) & ~1));
        for (int i = threadIdx.x; i < a.Wh * a.nsplit; i += TPB) sp[i] = a.split[i];
    }
}

__device__ __forceinline__ const uint32_t *split_of(const DpArgs &a, const uint16_t *tab) {
    if (!a.split_lds) return a.split;
    const int nt = a.p >= 2 ? a.Wq + a.n_rank : 0;
    return (const uint32_t *)(tab + ((nt + 1) & ~1));
}

// Eq. 1 rank of a mask of the k-1 colours other than the row's own.
__device__ __forceinline__ int rank_of(const DpArgs &a, const uint16_t *rk, uint32_t m) {
    return a.rank_direct ? rk[m] : rk[m & 255u] + rk[256 + (m >> 8) * 9 + __popc(m & 255u)];
}

// The (p-1)-subset masks of the passive-row entries q = 64*i + lane a lane
// reads (0 past the row).  They do not depend on the neighbour, so rows that
// fit CH chunks keep them in registers for the whole kernel.
template <int CH>
__device__ __forceinline__ void lane_masks(const DpArgs &a, const uint16_t *unr, int base,
                                           uint32_t (&msk)[CH]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int Lq = a.Wq * a.Bi;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const int q = base + kWave * i + lane;
        msk[i] = q < Lq ? unr[q >> a.sh] : 0u;
    }
}

// p >= 2: scatters the passive rows of neighbours [e0, e1) of row v (plane pl)
// into the LDS neighbour sum Nl.  Wavefront w of a team of W wavefronts takes
// neighbours e0 + w, e0 + w + W, ...; it loads NB neighbours' rows at a time,
// CH chunks of 64 contiguous uint64 each (NB * CH = 16 loads in flight per
// lane), and rows wider than CH chunks (BIG) are walked in groups of CH chunks.  Lane `ri` of
// every group of Bi lanes serves colouring pl*Bi + ri.  Each entry {col(u)} +
// T of a neighbour u lands on v's entry for the same set, re-ranked among the
// colours other than col(v); sets holding col(v) are skipped.  Distinct
// entries of one row land on distinct sets, so a wavefront's adds never
// collide; adds of different wavefronts meet in LDS atomics, whose returned
// old value gives the carry.
template <int CH, int NB, bool BIG, bool MOD>
__device__ __forceinline__ void scatter_wide(const Team &tm, const DpArgs &a, int64_t v, int pl, int64_t e0,
                                             int64_t e1, uint64_t *Nl, const uint16_t *unr,
                                             const uint16_t *rk, const uint32_t (&rmsk)[CH],
                                             uint64_t &m) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = tm.wave;
    const int waves = tm.waves;
    const int ri = lane & (a.Bi - 1);
    const int r = pl * a.Bi + ri;
    const int cv = a.col[v * a.B + r];
    const uint32_t vbit = 1u << cv;
    const int Lq = a.Wq * a.Bi;
    uint32_t carry = 0;
    // rows wider than CH chunks are walked a group of CH chunks at a time,
    // every neighbour's group before the next group, so a lane's set masks
    // are read once per group and row
    for (int base = 0; base < (BIG ? Lq : 1); base += kWave * CH) {
        uint32_t msk[CH];
        if (BIG) lane_masks<CH>(a, unr, base, msk);
        else {
#pragma unroll
            for (int i = 0; i < CH; ++i) msk[i] = rmsk[i];
        }
        for (int64_t eb = e0 + wave; eb < e1; eb += (int64_t)waves * NB) {
            int cu[NB];
            uint64_t x[NB][CH];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int64_t e = eb + (int64_t)b * waves;
                cu[b] = cv;                                // absent neighbour: skipped below
#pragma unroll
                for (int i = 0; i < CH; ++i) x[b][i] = 0;
                if (e < e1) {
                    const int u = __builtin_amdgcn_readfirstlane(a.ci[e]);
                    cu[b] = a.col[(int64_t)u * a.B + r];
                    const uint64_t *row = a.P + ((int64_t)pl * a.n + u) * Lq + base;
#pragma unroll
                    for (int i = 0; i < CH; ++i)
                        if (base + kWave * i + lane < Lq) x[b][i] = row[kWave * i + lane];
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (cu[b] == cv) continue;
                const uint32_t own = 1u << cu[b];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const uint64_t xv = x[b][i];
                    if (xv == 0) continue;
                    const uint32_t E = widen_at(msk[i], cu[b]) | own;
                    if (E & vbit) continue;
                    const int idx = rank_of(a, rk, narrow_at(E, cv));
                    unsigned long long *dst = (unsigned long long *)&Nl[(idx << a.sh) + ri];
                    const unsigned long long old = atomicAdd(dst, (unsigned long long)xv);
                    if ((uint64_t)old + xv < xv) {
                        if constexpr (MOD) put_back_wrap(dst, a.md.wrap);
                        else carry = 1;
                    }
                }
            }
        }
    }
    if (carry) m |= 1ull << r;
}

// The same scatter for rounds of many narrow rows (NB >= 4): the round's
// neighbour ids come in one load, every colour and row load of the round is
// issued before any is used, and the carries of up to eight adds are read
// together.
template <int CH, int NB, bool BIG, bool MOD>
__device__ __forceinline__ void scatter_narrow(const Team &tm, const DpArgs &a, int64_t v, int pl, int64_t e0,
                                             int64_t e1, uint64_t *Nl, const uint16_t *unr,
                                             const uint16_t *rk, const uint32_t (&rmsk)[CH],
                                             uint64_t &m) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = tm.wave;
    const int waves = tm.waves;
    const int ri = lane & (a.Bi - 1);
    const int r = pl * a.Bi + ri;
    const int cv = a.col[v * a.B + r];
    const uint32_t vbit = 1u << cv;
    const int Lq = a.Wq * a.Bi;
    uint32_t carry = 0;
    for (int64_t eb = e0 + wave; eb < e1; eb += (int64_t)waves * NB) {
        // lane b holds the b-th neighbour id of the round, broadcast to scalars
        int mine = -1;
        const int64_t el = eb + (int64_t)lane * waves;
        if (lane < NB && el < e1) mine = a.ci[el];
        int uid[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) uid[b] = __builtin_amdgcn_readlane(mine, b);
        for (int base = 0; base < (BIG ? Lq : 1); base += kWave * CH) {
            uint32_t msk[CH];
            if (BIG) lane_masks<CH>(a, unr, base, msk);
            else {
#pragma unroll
                for (int i = 0; i < CH; ++i) msk[i] = rmsk[i];
            }
            int cu[NB];
            uint64_t x[NB][CH];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                cu[b] = uid[b] >= 0 ? (int)a.col[(int64_t)uid[b] * a.B + r] : cv;
                const uint64_t *row = a.P + ((int64_t)pl * a.n + (uid[b] >= 0 ? uid[b] : 0)) * Lq + base;
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    x[b][i] = (uid[b] >= 0 && base + kWave * i + lane < Lq) ? row[kWave * i + lane] : 0;
            }
            // adds in groups of up to 8 whose carries are read after the group is issued
            constexpr int G = NB * CH < 8 ? NB * CH : 8;
#pragma unroll
            for (int f0 = 0; f0 < NB * CH; f0 += G) {
                uint64_t old[G];
                int tgt[G];
#pragma unroll
                for (int f = 0; f < G; ++f) {
                    const int b = (f0 + f) / CH, i = (f0 + f) % CH;
                    const uint32_t E = widen_at(msk[i], cu[b]) | (1u << cu[b]);
                    old[f] = 0;
                    tgt[f] = 0;
                    if (x[b][i] != 0 && cu[b] != cv && !(E & vbit)) {
                        const int idx = rank_of(a, rk, narrow_at(E, cv));
                        tgt[f] = (idx << a.sh) + ri;
                        old[f] = atomicAdd((unsigned long long *)&Nl[tgt[f]], (unsigned long long)x[b][i]);
                    } else {
                        x[b][i] = 0;
                    }
                }
#pragma unroll
                for (int f = 0; f < G; ++f) {
                    const uint64_t xv = x[(f0 + f) / CH][(f0 + f) % CH];
                    if (old[f] + xv < xv) {
                        if constexpr (MOD) put_back_wrap((unsigned long long *)&Nl[tgt[f]], a.md.wrap);
                        else carry = 1;
                    }
                }
            }
        }
    }
    if (carry) m |= 1ull << r;
}

// Rows of at most 16 sets (Wq <= 16) with Bi >= 4 interleaved colourings:
// each group of Bi lanes takes one neighbour (lane ri serving colouring
// pl*Bi + ri) and walks the row's Wq sets, so a load instruction reads 64/Bi
// neighbours' entries for one set; U rounds of neighbours are in flight.
// Groups of one wavefront may add to the same entry, so adds are LDS atomics
// (carry from the returned old value).
template <int U, bool MOD>
__device__ __forceinline__ void scatter_groups(const Team &tm, const DpArgs &a, int64_t v, int pl, int64_t e0,
                                               int64_t e1, uint64_t *Nl, const uint16_t *unr,
                                               const uint16_t *rk, uint64_t &m) {
    constexpr int kMaxW = 16;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = tm.wave;
    const int waves = tm.waves;
    const int ri = lane & (a.Bi - 1);
    const int grp = lane >> a.sh;
    const int groups = kWave >> a.sh;
    const int r = pl * a.Bi + ri;
    const int cv = a.col[v * a.B + r];
    const uint32_t vbit = 1u << cv;
    const int Lq = a.Wq * a.Bi;
    // neighbour e0 + wave + waves*(grp + groups*i): a short row spreads over
    // the wavefronts before it fills a wavefront's groups
    const int64_t round = (int64_t)waves * groups;
    uint32_t carry = 0;
    for (int64_t eb = e0 + wave + (int64_t)waves * grp; eb - (int64_t)waves * grp < e1; eb += round * U) {
        int u[U], cu[U];
        uint64_t x[U][kMaxW];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int64_t e = eb + t * round;
            u[t] = e < e1 ? a.ci[e] : -1;
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            cu[t] = u[t] >= 0 ? (int)a.col[(int64_t)u[t] * a.B + r] : cv;
            const uint64_t *row = a.P + ((int64_t)pl * a.n + (u[t] >= 0 ? u[t] : 0)) * Lq + ri;
#pragma unroll
            for (int j = 0; j < kMaxW; ++j)
                x[t][j] = (u[t] >= 0 && j < a.Wq) ? row[j << a.sh] : 0;
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const uint32_t own = 1u << cu[t];
#pragma unroll
            for (int j0 = 0; j0 < kMaxW; j0 += 8) {
                uint64_t old[8];
                int tgt[8];
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    const int j = j0 + f;
                    old[f] = 0;
                    tgt[f] = 0;
                    const uint32_t E = widen_at(unr[j < a.Wq ? j : 0], cu[t]) | own;
                    if (x[t][j] != 0 && cu[t] != cv && !(E & vbit)) {
                        const int idx = rank_of(a, rk, narrow_at(E, cv));
                        tgt[f] = (idx << a.sh) + ri;
                        old[f] = atomicAdd((unsigned long long *)&Nl[tgt[f]], (unsigned long long)x[t][j]);
                    } else {
                        x[t][j] = 0;
                    }
                }
#pragma unroll
                for (int f = 0; f < 8; ++f)
                    if (old[f] + x[t][j0 + f] < x[t][j0 + f]) {
                        if constexpr (MOD) put_back_wrap((unsigned long long *)&Nl[tgt[f]], a.md.wrap);
                        else carry = 1;
                    }
            }
        }
    }
    if (carry) m |= 1ull << r;
}

// Rounds of four or more narrow rows fetch their neighbour ids in one load
// and read the carries of a group of adds at once; rounds of one or two wide
// rows keep fewer registers live instead.
// CH == kGroupRows selects the lane-group scatter for rows of at most 16 sets.
template <int CH, int NB, bool BIG, bool MOD>
__device__ __forceinline__ void scatter_rows(const Team &tm, const DpArgs &a, int64_t v, int pl, int64_t e0,
                                             int64_t e1, uint64_t *Nl, const uint16_t *unr,
                                             const uint16_t *rk, const uint32_t (&rmsk)[CH],
                                             uint64_t &m) {
    if constexpr (CH == kGroupRows) scatter_groups<2, MOD>(tm, a, v, pl, e0, e1, Nl, unr, rk, m);
    else if constexpr (NB >= 4) scatter_narrow<CH, NB, BIG, MOD>(tm, a, v, pl, e0, e1, Nl, unr, rk, rmsk, m);
    else scatter_wide<CH, NB, BIG, MOD>(tm, a, v, pl, e0, e1, Nl, unr, rk, rmsk, m);
}

// p = 1: counts the colours of neighbours [e0, e1) of row v (plane pl): the
// neighbour sum of single-vertex tables is N'[v][{x}] = #{u : col(u) = x}, x
// renumbered among the colours other than col(v).  The team's threads are
// (neighbour slot, colouring) pairs.
__device__ __forceinline__ void count_colours(const Team &tm, const DpArgs &a, int64_t v, int pl,
                                              int64_t e0, int64_t e1, uint64_t *Nl) {
    const int ri = tm.tid & (a.Bi - 1);
    const int s = tm.tid >> a.sh;
    const int slots = tm.size >> a.sh;
    const int r = pl * a.Bi + ri;
    const int cv = a.col[v * a.B + r];
    for (int64_t e = e0 + s; e < e1; e += slots) {
        const int cu = a.col[(int64_t)a.ci[e] * a.B + r];
        if (cu != cv)
            atomicAdd((unsigned long long *)&Nl[((cu - (cu > cv)) << a.sh) + ri], 1ull);
    }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int mask) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, mask, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), mask, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// Output row of (v, pl): S[v] = N'[v] (a = 1) or, for every output set D and
// colouring, the sum over the nsplit pairs (Ia, Ip) of D of A[v][Ia] * N'[v][Ip].
// Each output entry is summed by a group of eg adjacent lanes (every eg-th
// pair), whose partial sums meet through cross-lane shuffles; all terms are
// non-negative, so a carry in any partial sum or in their combination means
// the exact sum reaches 2^64.  MOD: each lane keeps its sum of products
// exactly (a 128-bit word and a count of its carries) and reduces it mod p
// once; the lanes then meet by modular adds.  N32: the neighbour sums are
// colour counts (p = 1), below 2^32, so each product takes two 32-bit
// multiplies.
template <int AM, bool MOD, bool N32>
__device__ __forceinline__ void emit_row(const Team &tm, const DpArgs &a, int64_t v, int pl,
                                         const uint64_t *Nl, const uint64_t *Al, const uint32_t *split,
                                         uint64_t &m) {
    const int Ls = a.Wh * a.Bi;
    uint64_t *out = a.S + ((int64_t)pl * a.n + v) * Ls;
    if (AM == kActiveLeaf) {
        for (int q = tm.tid; q < Ls; q += tm.size) out[q] = Nl[q];
        return;
    }
    const uint64_t *Ar = AM == kActiveLds ? Al : a.A + ((int64_t)pl * a.n + v) * (int64_t)(a.Wa * a.Bi);
    const int g = tm.tid & (a.eg - 1);
    const int per = tm.size >> a.lg_eg;
    const int step = a.eg;
    const bool lean = a.nsplit >= kMad3Pairs;      // uniform: the step's form of the product
    for (int q0 = 0; q0 < Ls; q0 += per) {          // uniform over the block
        const int q = q0 + (tm.tid >> a.lg_eg);
        const int D = q >> a.sh, ri = q & (a.Bi - 1);
        uint64_t acc = 0;
        uint32_t ovf = 0;
        unsigned __int128 wlo = 0;                  // MOD: the lane's exact sum of products,
        uint64_t wtop = 0;                          // reduced once below
        if (q < Ls) {
            const uint32_t *sp = split + D;              // pair j at sp[j * Wh]
            int j = g;
            for (; j + 3 * step < a.nsplit; j += 4 * step) {
                uint32_t pr[4];
                uint64_t x[4], y[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) pr[i] = sp[(int64_t)(j + i * step) * a.Wh];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    x[i] = Ar[((pr[i] & 0xffffu) << a.sh) + ri];
                    y[i] = Nl[((pr[i] >> 16) << a.sh) + ri];
                }
                if constexpr (MOD && N32) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) wide_add_product_n32(wlo, wtop, x[i], (uint32_t)y[i]);
                } else if constexpr (MOD) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) wide_add_product(wlo, wtop, x[i], y[i]);
                } else if constexpr (N32) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc = mad_ovf_n32(acc, x[i], (uint32_t)y[i], ovf);
                } else if (lean) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc = mad_ovf3(acc, x[i], y[i], ovf);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc = mad_ovf(acc, x[i], y[i], ovf);
                }
            }
            for (; j < a.nsplit; j += step) {
                const uint32_t pr = sp[(int64_t)j * a.Wh];
                const uint64_t xa = Ar[((pr & 0xffffu) << a.sh) + ri], yn = Nl[((pr >> 16) << a.sh) + ri];
                if constexpr (MOD && N32) wide_add_product_n32(wlo, wtop, xa, (uint32_t)yn);
                else if constexpr (MOD) wide_add_product(wlo, wtop, xa, yn);
                else if constexpr (N32) acc = mad_ovf_n32(acc, xa, (uint32_t)yn, ovf);
                else acc = mad_ovf(acc, xa, yn, ovf);
            }
        }
        if constexpr (MOD) acc = mod_wide_fold(wlo, wtop, a.md);
        for (int o = 1; o < a.eg; o <<= 1) {
            const uint64_t y = shfl_xor_u64(acc, o);
            if constexpr (MOD) {
                acc = mod_add(acc, y, a.md);
            } else {
                ovf |= (uint32_t)__shfl_xor((int)ovf, o, kWave);
                const uint64_t t = acc + y;
                ovf |= (uint32_t)(t < y);
                acc = t;
            }
        }
        if (q < Ls && g == 0) {
            out[q] = acc;
            if (ovf) m |= 1ull << (pl * a.Bi + ri);
        }
    }
}

// One team per (plane, row) item, the grid striding over the items (rows are
// sorted by descending degree, so every team gets a similar mix).  The team is
// the workgroup, or (WAVE) each of its four wavefronts on its own row, for
// steps whose rows are small: a light row then needs no workgroup barrier and
// four times as many rows are in flight.  LDS per team: the neighbour-sum row
// N' (Wn * Bi) and the staged active row (Wa * Bi, AM == kActiveLds); then the
// index tables, shared by the workgroup.  CH = 0: p = 1.
template <int CH, int NB, bool BIG, int AM, bool WAVE, bool MOD, int TPB>
__global__ __launch_bounds__(TPB) void dp_row_kernel(DpArgs a) {
    constexpr bool HIST = CH == 0;
    constexpr int C = HIST ? 1 : CH;
    constexpr int kTeams = WAVE ? kWaves : 1;
    extern __shared__ uint64_t lds[];
    const Team tm = WAVE ? wave_team() : block_team<TPB>();
    const int Ln = a.Wn * a.Bi, La = a.Wa * a.Bi;
    const int region = Ln + (AM == kActiveLds ? La : 0);
    uint64_t *Nl = lds + (WAVE ? (int)(threadIdx.x >> 6) * region : 0);
    uint64_t *Al = Nl + Ln;
    uint16_t *tab = (uint16_t *)((char *)lds + a.tab_off);
    uint32_t msk[C];
    stage_tables<TPB>(a, tab);
    __syncthreads();
    if constexpr (!HIST && !BIG && CH != kGroupRows) lane_masks<C>(a, tab, 0, msk);
    const uint32_t *split = split_of(a, tab);
    const int64_t total = a.n * a.planes;
    uint64_t m = 0;
    for (int64_t it = (int64_t)blockIdx.x * kTeams + (WAVE ? (int)(threadIdx.x >> 6) : 0); it < total;
         it += (int64_t)gridDim.x * kTeams) {
        const int pl = (int)(it / a.n);
        const int64_t v = it - (int64_t)pl * a.n;
        const int sv = a.slot ? a.slot[v] : -1;
        if (sv >= 0) {
            const uint64_t *src = a.Npre + ((int64_t)pl * a.n_split + sv) * Ln;
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = src[q];
        } else {
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = 0;
        }
        if (AM == kActiveLds) {
            const uint64_t *src = a.A + ((int64_t)pl * a.n + v) * La;
            for (int q = tm.tid; q < La; q += tm.size) Al[q] = src[q];
        }
        team_sync<WAVE>();
        if (sv < 0) {
            if constexpr (HIST) count_colours(tm, a, v, pl, a.rp[v], a.rp[v + 1], Nl);
            else scatter_rows<C, NB, BIG, MOD>(tm, a, v, pl, a.rp[v], a.rp[v + 1], Nl, tab, tab + a.Wq, msk, m);
        }
        team_sync<WAVE>();
        if constexpr (MOD) {                     // the sums, known modulo p, into [0, p)
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = mod_fold(Nl[q], a.md);
            team_sync<WAVE>();
        }
        emit_row<AM, MOD, HIST>(tm, a, v, pl, Nl, Al, split, m);
        team_sync<WAVE>();                       // LDS is reused by the next item
    }
    flush_flags(m, a.flags);
}

// The root step of a template on all k colours, (k, 1, k-1): the single-vertex
// root joins a passive child that holds every other colour, so the output row
// is one set (all k colours) and the neighbour sum one entry (the k-1 colours
// other than col(v)).  Of a neighbour u's row only the entry that leaves out
// col(v) adds to it: in u's space (the colours other than col(u), renumbered
// 0..k-2) the (k-2)-subset that misses col(v)'s index x, whose Eq. 1 rank is
// k-2-x; a neighbour with col(u) = col(v) adds nothing.  So a visit reads one
// word per colouring, not the whole row.  One wavefront per (plane, row):
// groups of Bi lanes take the row's neighbours in turn, lane ri of a group
// serving colouring pl*Bi + ri, and the groups meet through shuffles (carry
// flags, or modular adds).  Visits are cheap enough that rows above the
// segment size are summed here too: the step has no split pre-pass.

template <bool MOD>
__global__ __launch_bounds__(kBlock) void dp_root_kernel(DpArgs a) {
    constexpr int kTeams = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int ri = lane & (a.Bi - 1);
    const int grp = lane >> a.sh, groups = kWave >> a.sh;
    const int k2 = a.Wq - 1;                     // k - 2: a row of P holds k - 1 entries
    const int64_t total = a.n * a.planes;
    uint64_t m = 0;
    for (int64_t it = (int64_t)blockIdx.x * kTeams + (int)(threadIdx.x >> 6); it < total;
         it += (int64_t)gridDim.x * kTeams) {
        const int pl = (int)(it / a.n);
        const int64_t v = it - (int64_t)pl * a.n;
        const int r = pl * a.Bi + ri;
        uint64_t acc = 0;
        uint32_t carry = 0;
        const int cv = a.col[v * a.B + r];
        const int64_t e1 = a.rp[v + 1];
        for (int64_t e = a.rp[v] + grp; e < e1; e += groups) {
            const int u = a.ci[e];
            const int cu = a.col[(int64_t)u * a.B + r];
            if (cu == cv) continue;
            const int x = cv - (cv > cu);
            const uint64_t y = a.P[(((int64_t)pl * a.n + u) * a.Wq + (k2 - x)) * a.Bi + ri];
            if constexpr (MOD) {
                acc = mod_add(acc, y, a.md);
            } else {
                const uint64_t t = acc + y;
                carry |= (uint32_t)(t < y);
                acc = t;
            }
        }
        for (int o = a.Bi; o < kWave; o <<= 1) {
            const uint64_t y = shfl_xor_u64(acc, o);
            if constexpr (MOD) {
                acc = mod_add(acc, y, a.md);
            } else {
                carry |= (uint32_t)__shfl_xor((int)carry, o, kWave);
                const uint64_t t = acc + y;
                carry |= (uint32_t)(t < y);
                acc = t;
            }
        }
        if (grp == 0) {
            a.S[((int64_t)pl * a.n + v) * a.Bi + ri] = acc;
            if (carry) m |= 1ull << r;
        }
    }
    flush_flags(m, a.flags);
}

// Split rows: one workgroup per (plane, row, segment of `seg` neighbours)
// item; the segment's sum is built in LDS as in the row kernel and added into
// Npre with global atomics (carry from the returned old value).
template <int CH, int NB, bool BIG, bool MOD, int TPB>
__global__ __launch_bounds__(TPB) void dp_split_kernel(DpArgs a) {
    constexpr bool HIST = CH == 0;
    constexpr int C = HIST ? 1 : CH;
    extern __shared__ uint64_t lds[];
    uint64_t *Nl = lds;
    uint16_t *tab = (uint16_t *)((char *)lds + a.tab_off);
    uint32_t msk[C];
    if constexpr (!HIST) {
        stage_tables<TPB>(a, tab);
        __syncthreads();
        if constexpr (!BIG && CH != kGroupRows) lane_masks<C>(a, tab, 0, msk);
    }
    const int Ln = a.Wn * a.Bi;
    const int64_t total = a.n_items * a.planes;
    uint64_t m = 0;
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int pl = (int)(it / a.n_items);
        const int2 item = a.items[it - (int64_t)pl * a.n_items];
        const int64_t v = item.x;
        const int64_t r1 = a.rp[v + 1];
        const int64_t e0 = a.rp[v] + (int64_t)item.y * a.seg;
        const int64_t e1 = e0 + a.seg < r1 ? e0 + a.seg : r1;
        for (int q = threadIdx.x; q < Ln; q += TPB) Nl[q] = 0;
        __syncthreads();
        if constexpr (HIST) count_colours(block_team<TPB>(), a, v, pl, e0, e1, Nl);
        else scatter_rows<C, NB, BIG, MOD>(block_team<TPB>(), a, v, pl, e0, e1, Nl, tab, tab + a.Wq, msk, m);
        __syncthreads();
        unsigned long long *dst =
            (unsigned long long *)a.Npre + ((int64_t)pl * a.n_split + a.slot[v]) * Ln;
        for (int q = threadIdx.x; q < Ln; q += TPB) {
            const uint64_t x = Nl[q];
            if (x == 0) continue;
            const unsigned long long old = atomicAdd(dst + q, (unsigned long long)x);
            if ((uint64_t)old + x < x) {
                if constexpr (MOD) put_back_wrap(dst + q, a.md.wrap);
                else m |= 1ull << (pl * a.Bi + (q & (a.Bi - 1)));
            }
        }
        __syncthreads();
    }
    flush_flags(m, a.flags);
}

// ------------------------------------------------------------------ chains of single-vertex attaches

struct ChainStepArgs {
    const uint32_t *split;        // a >= 2: the (k-1, h-1, a-1) split table
    int Wh, nsplit, eg, lg_eg;
    int lin, lout;                // exact multi-limb chain: limbs of the step's input and output rows
};

struct ChainArgs {
    DpArgs d;                     // graph, colours, interleave, split rows, flags, modulus
    int steps, a0, wmax, k1, Wa0;
    const uint64_t *A;
    uint64_t *S;
    ChainStepArgs st[kMaxChainSteps];
};

// One chain step's output row: for every output set D and colouring, the sum
// over the nsplit pairs (Ia, {x}) of D (the split table, read through the
// caches) of cur[Ia] * N'[x], N' the row's neighbour colour counts (below
// 2^32: the two-multiply product); four pairs per lane are issued together,
// and a group of eg lanes per entry meets as in emit_row.  `out` is the next
// LDS row, or the step's table in global memory for the chain's last step.
template <bool MOD>
__device__ __forceinline__ void chain_emit(const Team &tm, const DpArgs &a, const ChainStepArgs &cs, int pl,
                                           const uint64_t *cur, const uint64_t *Nl, uint64_t *out, uint64_t &m) {
    const int Ls = cs.Wh * a.Bi;
    const int g = tm.tid & (cs.eg - 1);
    const int per = tm.size >> cs.lg_eg;
    const int step = cs.eg;
    for (int q0 = 0; q0 < Ls; q0 += per) {          // uniform over the team
        const int q = q0 + (tm.tid >> cs.lg_eg);
        const int D = q >> a.sh, ri = q & (a.Bi - 1);
        uint64_t acc = 0;
        uint32_t ovf = 0;
        unsigned __int128 wlo = 0;
        uint64_t wtop = 0;
        if (q < Ls) {
            const uint32_t *sp = cs.split + D;           // pair j at sp[j * Wh]
            int j = g;
            for (; j + 3 * step < cs.nsplit; j += 4 * step) {
                uint32_t pr[4];
                uint64_t x[4];
                uint32_t y[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) pr[i] = sp[(int64_t)(j + i * step) * cs.Wh];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    x[i] = cur[((pr[i] & 0xffffu) << a.sh) + ri];
                    y[i] = (uint32_t)Nl[((pr[i] >> 16) << a.sh) + ri];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (MOD) wide_add_product_n32(wlo, wtop, x[i], y[i]);
                    else acc = mad_ovf_n32(acc, x[i], y[i], ovf);
                }
            }
            for (; j < cs.nsplit; j += step) {
                const uint32_t pr = sp[(int64_t)j * cs.Wh];
                const uint64_t xa = cur[((pr & 0xffffu) << a.sh) + ri];
                const uint32_t yn = (uint32_t)Nl[((pr >> 16) << a.sh) + ri];
                if constexpr (MOD) wide_add_product_n32(wlo, wtop, xa, yn);
                else acc = mad_ovf_n32(acc, xa, yn, ovf);
            }
        }
        if constexpr (MOD) acc = mod_wide_fold(wlo, wtop, a.md);
        for (int o = 1; o < cs.eg; o <<= 1) {
            const uint64_t y = shfl_xor_u64(acc, o);
            if constexpr (MOD) {
                acc = mod_add(acc, y, a.md);
            } else {
                ovf |= (uint32_t)__shfl_xor((int)ovf, o, kWave);
                const uint64_t t = acc + y;
                ovf |= (uint32_t)(t < y);
                acc = t;
            }
        }
        if (q < Ls && g == 0) {
            out[q] = acc;
            if (ovf) m |= 1ull << (pl * a.Bi + ri);
        }
    }
}

// A chain of steps whose passive children are single vertices, one team per
// (plane, row) item as in dp_row_kernel: the row's neighbour colour counts N'
// (from the split pre-pass for rows above the segment size), then every step
// of the chain on the row, its output in LDS (two rows used in turn), and the
// last step's output written to its table.  For a0 = 1 the first step's
// output is N' itself.  LDS per team: N' (k1 * Bi), then two rows of wmax * Bi.
template <bool WAVE, bool MOD, int TPB>
__global__ __launch_bounds__(TPB) void dp_chain_kernel(ChainArgs c) {
    constexpr int kTeams = WAVE ? TPB / kWave : 1;
    extern __shared__ uint64_t lds[];
    const DpArgs &a = c.d;
    const Team tm = WAVE ? wave_team() : block_team<TPB>();
    const int Ln = c.k1 * a.Bi, Lw = c.wmax * a.Bi;
    uint64_t *Nl = lds + (WAVE ? (int)(threadIdx.x >> 6) * (Ln + 2 * Lw) : 0);
    uint64_t *rows[2] = {Nl + Ln, Nl + Ln + Lw};
    const int64_t total = a.n * a.planes;
    uint64_t m = 0;
    for (int64_t it = (int64_t)blockIdx.x * kTeams + (WAVE ? (int)(threadIdx.x >> 6) : 0); it < total;
         it += (int64_t)gridDim.x * kTeams) {
        const int pl = (int)(it / a.n);
        const int64_t v = it - (int64_t)pl * a.n;
        const int sv = a.slot ? a.slot[v] : -1;
        if (sv >= 0) {
            const uint64_t *src = a.Npre + ((int64_t)pl * a.n_split + sv) * Ln;
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = src[q];
        } else {
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = 0;
        }
        if (c.a0 > 1) {
            const int La = c.Wa0 * a.Bi;
            const uint64_t *src = c.A + ((int64_t)pl * a.n + v) * La;
            for (int q = tm.tid; q < La; q += tm.size) rows[0][q] = src[q];
        }
        team_sync<WAVE>();
        if (sv < 0) count_colours(tm, a, v, pl, a.rp[v], a.rp[v + 1], Nl);
        team_sync<WAVE>();
        const uint64_t *cur = c.a0 > 1 ? rows[0] : Nl;   // a0 = 1: the first output is N'
        int next = c.a0 > 1 ? 1 : 0;
        for (int i = c.a0 > 1 ? 0 : 1; i < c.steps; ++i) {
            const ChainStepArgs &cs = c.st[i];
            uint64_t *out = i == c.steps - 1 ? c.S + ((int64_t)pl * a.n + v) * (int64_t)(cs.Wh * a.Bi) : rows[next];
            chain_emit<MOD>(tm, a, cs, pl, cur, Nl, out, m);
            team_sync<WAVE>();                   // the output is the next step's input; LDS is
            cur = out;                           // reused by the next item after the last step
            next ^= 1;
        }
    }
    flush_flags(m, a.flags);
}

// Exact counts of a template that is one chain from a single vertex (a star
// rooted at its centre): every entry is kept as little-endian 64-bit limbs,
// so no count is reduced modulo anything.  A step's entries count colourful
// maps of a sub-star rooted at the row's vertex, so the largest homomorphism
// count of that sub-star at any vertex bounds them; each step keeps the
// fewest limbs (1..4) that hold its bound, so early steps stay one word
// wide.  A carry out of a step's top limb (impossible under the bounds) sets
// the colouring's flag.

// acc (LO limbs) += x (LI <= LO limbs) * y for a 32-bit y; returns the carry
// out of the top limb.
template <int LI, int LO>
__device__ __forceinline__ uint64_t wide_mad_n32(uint64_t (&acc)[LO], const uint64_t *x, uint32_t y) {
    uint64_t carry = 0;
#pragma unroll
    for (int l = 0; l < LI; ++l) {
        const unsigned __int128 pr = (unsigned __int128)x[l] * y + carry;   // < 2^96 + 2^64
        const uint64_t lo = (uint64_t)pr;
        carry = (uint64_t)(pr >> 64);
        acc[l] += lo;
        carry += acc[l] < lo;
    }
#pragma unroll
    for (int l = LI; l < LO; ++l) {
        acc[l] += carry;
        carry = acc[l] < carry;
    }
    return carry;
}

// One step of the exact chain: out[q] (LO limbs) = the sum over the members x
// of output set D of cur[D - {x}] (LI limbs) * N'[x], with the pairs from the
// pair-major split table; a group of eg lanes per entry meets through
// shuffles, limb by limb with carries.
template <int LI, int LO>
__device__ __forceinline__ void chain_emit_wide(const Team &tm, const DpArgs &a, const ChainStepArgs &cs, int pl,
                                                const uint64_t *cur, const uint64_t *Nl, uint64_t *out,
                                                uint64_t &m) {
    const int Ls = cs.Wh * a.Bi;
    const int g = tm.tid & (cs.eg - 1);
    const int per = tm.size >> cs.lg_eg;
    for (int q0 = 0; q0 < Ls; q0 += per) {          // uniform over the team
        const int q = q0 + (tm.tid >> cs.lg_eg);
        const int D = q >> a.sh, ri = q & (a.Bi - 1);
        uint64_t acc[LO];
#pragma unroll
        for (int l = 0; l < LO; ++l) acc[l] = 0;
        uint64_t top = 0;
        if (q < Ls) {
            const uint32_t *sp = cs.split + D;
            for (int j = g; j < cs.nsplit; j += cs.eg) {
                const uint32_t pr = sp[(int64_t)j * cs.Wh];
                const uint64_t *xa = cur + (int64_t)(((pr & 0xffffu) << a.sh) + ri) * LI;
                const uint32_t yn = (uint32_t)Nl[((pr >> 16) << a.sh) + ri];
                top |= wide_mad_n32<LI, LO>(acc, xa, yn);
            }
        }
        for (int o = 1; o < cs.eg; o <<= 1) {
            uint64_t c = 0;
#pragma unroll
            for (int l = 0; l < LO; ++l) {
                const uint64_t y = shfl_xor_u64(acc[l], o);
                const uint64_t t = acc[l] + y;
                const uint64_t c1 = t < y;
                acc[l] = t + c;
                c = c1 + (acc[l] < t);
            }
            top |= c | shfl_xor_u64(top, o);
        }
        if (q < Ls && g == 0) {
#pragma unroll
            for (int l = 0; l < LO; ++l) out[(int64_t)q * LO + l] = acc[l];
            if (top) m |= 1ull << (pl * a.Bi + ri);
        }
    }
}

template <int LI, int LO>
__device__ __forceinline__ void chain_emit_wide_if(const Team &tm, const DpArgs &a, const ChainStepArgs &cs,
                                                   int pl, const uint64_t *cur, const uint64_t *Nl, uint64_t *out,
                                                   uint64_t &m) {
    if (cs.lin == LI && cs.lout == LO) chain_emit_wide<LI, LO>(tm, a, cs, pl, cur, Nl, out, m);
}

// The exact chain kernel: as dp_chain_kernel for a0 = 1, step i's rows
// holding st[i].lout limbs per entry (st[0]: the colour counts N', one limb).
// LDS per team: N' (k1 * Bi), then two rows of wmax * Bi words (wmax: the
// widest intermediate row in entries times limbs).
template <bool WAVE, int TPB>
__global__ __launch_bounds__(TPB) void dp_chain_wide_kernel(ChainArgs c) {
    constexpr int kTeams = WAVE ? TPB / kWave : 1;
    extern __shared__ uint64_t lds[];
    const DpArgs &a = c.d;
    const Team tm = WAVE ? wave_team() : block_team<TPB>();
    const int Ln = c.k1 * a.Bi, Lw = c.wmax * a.Bi;
    uint64_t *Nl = lds + (WAVE ? (int)(threadIdx.x >> 6) * (Ln + 2 * Lw) : 0);
    uint64_t *rows[2] = {Nl + Ln, Nl + Ln + Lw};
    const int64_t total = a.n * a.planes;
    uint64_t m = 0;
    for (int64_t it = (int64_t)blockIdx.x * kTeams + (WAVE ? (int)(threadIdx.x >> 6) : 0); it < total;
         it += (int64_t)gridDim.x * kTeams) {
        const int pl = (int)(it / a.n);
        const int64_t v = it - (int64_t)pl * a.n;
        const int sv = a.slot ? a.slot[v] : -1;
        if (sv >= 0) {
            const uint64_t *src = a.Npre + ((int64_t)pl * a.n_split + sv) * Ln;
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = src[q];
        } else {
            for (int q = tm.tid; q < Ln; q += tm.size) Nl[q] = 0;
        }
        team_sync<WAVE>();
        if (sv < 0) count_colours(tm, a, v, pl, a.rp[v], a.rp[v + 1], Nl);
        team_sync<WAVE>();
        // the first step's output is N' itself (one limb)
        const uint64_t *cur = Nl;
        int next = 0;
        for (int i = 1; i < c.steps; ++i) {
            const ChainStepArgs &cs = c.st[i];
            uint64_t *out = i == c.steps - 1
                                ? c.S + ((int64_t)pl * a.n + v) * (int64_t)(cs.Wh * a.Bi) * cs.lout
                                : rows[next];
            chain_emit_wide_if<1, 1>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<1, 2>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<1, 3>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<1, 4>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<2, 2>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<2, 3>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<2, 4>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<3, 3>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<3, 4>(tm, a, cs, pl, cur, Nl, out, m);
            chain_emit_wide_if<4, 4>(tm, a, cs, pl, cur, Nl, out, m);
            team_sync<WAVE>();
            cur = out;
            next ^= 1;
        }
    }
    flush_flags(m, a.flags);
}

// grid: (blocks, B): X[r][0..L] += the sum of colouring r's n*W entries of S
// (L limbs each), exactly: per thread, then a block tree, then limb-by-limb
// atomics whose carries go into the next limb.
template <int L>
__global__ __launch_bounds__(kBlock) void reduce_wide_kernel(int64_t n, const uint64_t *__restrict__ S, int W,
                                                            int Bi, unsigned long long *__restrict__ X) {
    __shared__ uint64_t part[L + 1][kBlock];
    const int r = blockIdx.y;
    const int pl = r / Bi, ri = r - pl * Bi;
    const int64_t total = n * W;
    const uint64_t *base = S + ((int64_t)pl * total * Bi + ri) * L;
    uint64_t acc[L + 1];
#pragma unroll
    for (int l = 0; l <= L; ++l) acc[l] = 0;
    auto add = [&](const uint64_t *x) {
        uint64_t c = 0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const uint64_t t = acc[l] + x[l];
            const uint64_t c1 = t < x[l];
            acc[l] = t + c;
            c = c1 + (acc[l] < t);
        }
        acc[L] += c;
    };
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        uint64_t x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = base[i * Bi * L + l];
        add(x);
    }
#pragma unroll
    for (int l = 0; l <= L; ++l) part[l][threadIdx.x] = acc[l];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            uint64_t c = 0;
#pragma unroll
            for (int l = 0; l <= L; ++l) {
                const uint64_t y = part[l][threadIdx.x + w];
                const uint64_t t = part[l][threadIdx.x] + y;
                const uint64_t c1 = t < y;
                part[l][threadIdx.x] = t + c;
                c = c1 + (part[l][threadIdx.x] < t);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t c = 0;
        for (int l = 0; l <= L; ++l) {
            const uint64_t x = part[l][0];
            const uint64_t x2 = x + c;
            c = x2 < x;
            if (x2 == 0) continue;
            const unsigned long long old = atomicAdd(&X[(int64_t)r * (L + 1) + l], (unsigned long long)x2);
            c += (uint64_t)old + x2 < x2;
        }
    }
}

// ------------------------------------------------------------------ root reduction

// grid: (blocks, B); block y = colouring r = pl*Bi + ri sums the n*W entries of
// that colouring (stride Bi inside plane pl).  MOD: the entries are residues
// mod md.p and X[r] ends congruent to their sum.
template <bool MOD>
__global__ __launch_bounds__(kBlock) void reduce_kernel(int64_t n, const uint64_t *__restrict__ S,
                                                       int W, int Bi, Modulus md,
                                                       unsigned long long *__restrict__ X,
                                                       unsigned long long *__restrict__ flags) {
    __shared__ uint64_t part[kBlock];
    __shared__ uint32_t cpart[kBlock];
    const int r = blockIdx.y;
    const int pl = r / Bi, ri = r - pl * Bi;
    const int64_t total = n * W;
    const uint64_t *base = S + (int64_t)pl * total * Bi + ri;
    uint64_t acc = 0;
    uint32_t carry = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const uint64_t x = base[i * Bi];
        if constexpr (MOD) {
            acc = mod_add(acc, x, md);
        } else {
            const uint64_t s = acc + x;
            carry |= s < x;
            acc = s;
        }
    }
    part[threadIdx.x] = acc;
    cpart[threadIdx.x] = carry;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const uint64_t x = part[threadIdx.x + w];
            if constexpr (MOD) {
                part[threadIdx.x] = mod_add(part[threadIdx.x], x, md);
            } else {
                const uint64_t s = part[threadIdx.x] + x;
                cpart[threadIdx.x] |= cpart[threadIdx.x + w] | (s < x);
                part[threadIdx.x] = s;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long old = atomicAdd(&X[r], (unsigned long long)part[0]);
        const bool wrapped = (uint64_t)old + part[0] < (uint64_t)old;
        if constexpr (MOD) {
            if (wrapped) put_back_wrap(&X[r], md.wrap);
        } else if (cpart[0] || wrapped) {
            atomicOr(flags, 1ull << r);
        }
    }
}

// ------------------------------------------------------------------ homomorphism bound

// Homomorphisms of the sub-template into the graph rooted at each row, in
// double: S[v] = A[v] * sum over neighbours u of P[u] (A or P NULL: the
// single-vertex sub-template, 1 at every row).  One wavefront per row.
__global__ __launch_bounds__(kBlock) void hom_step_kernel(int64_t n, const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ A,
                                                         const double *__restrict__ P,
                                                         double *__restrict__ S) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); v < n; v += waves) {
        const int64_t e0 = rp[v], e1 = rp[v + 1];
        double acc = 0;
        if (P) {
            for (int64_t e = e0 + lane; e < e1; e += kWave) acc += P[ci[e]];
            for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        } else {
            acc = (double)(e1 - e0);
        }
        if (lane == 0) S[v] = A ? A[v] * acc : acc;
    }
}

// out[0] += sum of S[0..n).
__global__ __launch_bounds__(kBlock) void hom_sum_kernel(int64_t n, const double *__restrict__ S,
                                                        double *__restrict__ out) {
    __shared__ double part[kBlock];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        acc += S[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, part[0]);
}

// The largest of S[0..n) into *out; non-negative doubles order as their bit
// patterns, so the blocks meet in an unsigned 64-bit atomic max.
__global__ __launch_bounds__(kBlock) void hom_max_kernel(int64_t n, const double *__restrict__ S,
                                                        unsigned long long *__restrict__ out) {
    __shared__ double part[kBlock];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        acc = fmax(acc, S[i]);
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(part[0]));
}

// ------------------------------------------------------------------ vector-ALU roof

// The multiply-add's arithmetic alone: each thread runs kProbeChains
// independent chains of `iters` exact multiply-adds with overflow detection
// (FORM 0: the 128-bit product, mad_ovf; 1: three 32-bit multiplies,
// mad_ovf3; 2: a 32-bit second operand, mad_ovf_n32) on register operands, and
// writes its sums and flag so that nothing is folded away.
constexpr int kProbeChains = 8;

template <int FORM>
__global__ __launch_bounds__(kBlock) void valu_probe_kernel(uint64_t seed, int iters,
                                                           unsigned long long *__restrict__ out) {
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t a[kProbeChains], acc[kProbeChains];
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j) {
        a[j] = (seed ^ (tid * 0x9E3779B97F4A7C15ull)) + (uint64_t)j * 0xBF58476D1CE4E5B9ull;
        acc[j] = 0;
    }
    uint64_t b = seed + tid;
    uint32_t ovf = 0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kProbeChains; ++j) {
            if constexpr (FORM == 0) acc[j] = mad_ovf(acc[j], a[j], b, ovf);
            else if constexpr (FORM == 1) acc[j] = mad_ovf3(acc[j], a[j], b, ovf);
            else acc[j] = mad_ovf_n32(acc[j], a[j], (uint32_t)b, ovf);
        }
        b += 0x94D049BB133111EBull;
    }
    uint64_t s = ovf;
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j) s += acc[j];
    out[tid] = s;
}

__global__ __launch_bounds__(kBlock) void zero_kernel(uint64_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0;
}

// Instantiation launched last by this thread (for launch tracing).
thread_local char t_last_kernel[96];

void name_kernel(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void name_kernel(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_last_kernel, sizeof t_last_kernel, fmt, ap);
    va_end(ap);
}

const char *tf(bool b) { return b ? "true" : "false"; }

int log2_exact(int x) {
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

// Workgroups that stay resident on the chip for a given dynamic LDS size.
int64_t resident_blocks(int lds_bytes, int tpb = kBlock) {
    const int per_cu = std::max(1, std::min(kMaxBlocksPerCU * kBlock / tpb, kLdsPerCU / std::max(lds_bytes, 1)));
    return (int64_t)per_cu * kCUs;
}

template <typename K>
hipError_t allow_lds(K kernel, int bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kLdsPerCU);
}

// Split-table entries staged in LDS (0: read from global memory).
int split_lds_words(const StepShape &s) {
    const int64_t w = (int64_t)s.Wh * s.nsplit;
    return s.amode != kActiveLeaf && s.a >= 2 && w <= kSplitLdsMax ? (int)w : 0;
}

// p = 2^w - c with 61 <= w <= 63 and c odd, c <= 2^16: the forms mod_fold
// reduces in three folds.
bool make_modulus(uint64_t p, Modulus &m) {
    m = Modulus{};
    if (p == 0) return true;
    int w = 64;
    while (w > 0 && !((p >> (w - 1)) & 1)) --w;      // p < 2^w
    if (w < 61 || w > 63) return false;
    const uint64_t c = (1ull << w) - p;
    if (c == 0 || c > (1ull << 16) || !(c & 1)) return false;
    m.p = p; m.c = c; m.w = w;
    m.wrap = (uint64_t)(((unsigned __int128)1 << 64) % p);
    return true;
}

DpArgs make_args(const GraphBins &g, const StepShape &s, const StepTables &t, const uint8_t *col,
                 const uint64_t *P, const uint64_t *A, const uint64_t *Npre, uint64_t *S,
                 unsigned long long *flags, int teams, int tpb = kBlock) {
    DpArgs a{};
    a.rp = g.row_ptr; a.ci = g.col_idx; a.col = col; a.n = g.n;
    a.B = s.B; a.Bi = s.Bi; a.sh = log2_exact(s.Bi); a.planes = s.B / s.Bi;
    a.p = s.p; a.Wq = s.Wq; a.Wn = s.Wn; a.Wa = s.Wa; a.Wh = s.Wh; a.nsplit = s.nsplit;
    // lanes per output entry: the power of two that shortens the longest
    // chain (rounds of outputs times pairs per lane)
    a.eg = 1; a.lg_eg = 0;
    {
        const int Ls = s.Wh * s.Bi;
        const int threads = tpb / teams;                 // threads building one row
        int64_t best = -1;
        for (int lg = 0, G = 1; G <= kWave; ++lg, G *= 2) {
            if (G > 1 && G / 2 >= s.nsplit) break;
            const int64_t rounds = (Ls + (threads / G) - 1) / (threads / G);
            const int64_t chain = rounds * (((int64_t)s.nsplit + G - 1) / G + 2 * lg);
            if (best < 0 || chain < best) { best = chain; a.eg = G; a.lg_eg = lg; }
        }
    }
    a.split = t.split; a.unrank = t.unrank; a.rank = t.rank; a.n_rank = t.n_rank;
    a.rank_direct = s.k - 1 <= kDirectRankBits;
    a.P = P; a.A = A; a.S = S; a.Npre = const_cast<uint64_t *>(Npre);
    a.slot = g.n_split ? g.slot : nullptr; a.n_split = g.n_split;
    a.items = g.split_items; a.n_items = g.n_split_items; a.seg = g.seg;
    a.tab_off = 8 * teams * (s.Wn * s.Bi + (s.amode == kActiveLds ? s.Wa * s.Bi : 0));
    a.split_lds = s.amode != kActiveLeaf && split_lds_words(s) > 0;
    a.flags = flags;
    make_modulus(s.mod, a.md);
    return a;
}

template <int CH, int NB, bool BIG, int AM, bool WAVE, bool MOD, int TPB = kBlock>
hipError_t row_launch(const DpArgs &a, int lds, hipStream_t st) {
    hipError_t e = allow_lds(dp_row_kernel<CH, NB, BIG, AM, WAVE, MOD, TPB>, lds);
    if (e != hipSuccess) return e;
    const int64_t teams = WAVE ? kWaves : 1;
    const int64_t blocks = std::min<int64_t>((a.n * a.planes + teams - 1) / teams, 2 * resident_blocks(lds, TPB));
    name_kernel("dp_row_kernel<%d, %d, %s, %d, %s, %s, %d>", CH, NB, tf(BIG), AM, tf(WAVE), tf(MOD), TPB);
    dp_row_kernel<CH, NB, BIG, AM, WAVE, MOD, TPB><<<dim3((unsigned)blocks), dim3(TPB), lds, st>>>(a);
    return hipGetLastError();
}

template <int CH, int NB, bool BIG, bool MOD, int TPB = kBlock>
hipError_t split_launch(const DpArgs &a, int lds, hipStream_t st) {
    hipError_t e = allow_lds(dp_split_kernel<CH, NB, BIG, MOD, TPB>, lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>(a.n_items * a.planes, 2 * resident_blocks(lds, TPB));
    name_kernel("dp_split_kernel<%d, %d, %s, %s, %d>", CH, NB, tf(BIG), tf(MOD), TPB);
    dp_split_kernel<CH, NB, BIG, MOD, TPB><<<dim3((unsigned)blocks), dim3(TPB), lds, st>>>(a);
    return hipGetLastError();
}

// Rows walked in groups of chunks whose LDS leaves few workgroups per CU.
bool wide_workgroup(const StepShape &s, int lds, bool wave);

// Chunks of 64 uint64 per passive row, rounded up to a power of two (0 for
// p = 1, 32 for rows wider than 16 chunks, walked in groups of 16), or
// kGroupRows (when `groups`) for rows of at most 16 sets with 4 or more
// interleaved colourings.
int row_chunks(const StepShape &s, bool groups) {
    if (s.p < 2) return 0;
    if (groups && s.Wq <= 16 && s.Bi >= 4) return kGroupRows;
    const int ch = (s.Wq * s.Bi + kWave - 1) / kWave;
    int c = 1;
    while (c < ch && c < 32) c *= 2;
    return c;
}

// The row kernels keep the chunked scatter for narrow rows too: a light row's
// few neighbours spread over more lanes that way.
template <int AM, bool WAVE, bool MOD>
hipError_t row_dispatch(const StepShape &s, const DpArgs &a, int lds, hipStream_t st) {
    switch (row_chunks(s, false)) {
    case 0: return row_launch<0, 1, false, AM, WAVE, MOD>(a, lds, st);
    case 1: return row_launch<1, 8, false, AM, WAVE, MOD>(a, lds, st);
    case 2: return row_launch<2, 8, false, AM, WAVE, MOD>(a, lds, st);
    case 4: return row_launch<4, 4, false, AM, WAVE, MOD>(a, lds, st);
    case 8: return row_launch<8, 2, false, AM, WAVE, MOD>(a, lds, st);
    case 16: return row_launch<16, 1, false, AM, WAVE, MOD>(a, lds, st);
    default:
        if constexpr (!WAVE)
            if (lds > kWideLds) return row_launch<16, 1, true, AM, WAVE, MOD, kBlockWide>(a, lds, st);
        return row_launch<16, 1, true, AM, WAVE, MOD>(a, lds, st);
    }
}

template <bool MOD>
hipError_t split_dispatch(const StepShape &s, const DpArgs &a, int lds, hipStream_t st) {
    switch (row_chunks(s, true)) {
    case 0: return split_launch<0, 1, false, MOD>(a, lds, st);
    case kGroupRows: return split_launch<kGroupRows, 1, false, MOD>(a, lds, st);
    case 1: return split_launch<1, 8, false, MOD>(a, lds, st);
    case 2: return split_launch<2, 8, false, MOD>(a, lds, st);
    case 4: return split_launch<4, 4, false, MOD>(a, lds, st);
    case 8: return split_launch<8, 2, false, MOD>(a, lds, st);
    case 16: return split_launch<16, 1, false, MOD>(a, lds, st);
    default:
        if (lds > kWideLds) return split_launch<16, 1, true, MOD, kBlockWide>(a, lds, st);
        return split_launch<16, 1, true, MOD>(a, lds, st);
    }
}

bool wide_workgroup(const StepShape &s, int lds, bool wave) {
    return !wave && row_chunks(s, false) > 16 && lds > kWideLds;
}

bool shape_ok(const StepShape &s) {
    Modulus m;
    return s.Bi >= 1 && s.Bi <= kWave && (s.Bi & (s.Bi - 1)) == 0 && s.B % s.Bi == 0 &&
           s.Wn >= 1 && s.Wh >= 1 && (s.p < 2 || s.Wq >= 1) && make_modulus(s.mod, m);
}

}  // namespace

bool mod_supported(uint64_t p) {
    Modulus m;
    return p != 0 && make_modulus(p, m);
}

const char *last_kernel_name() { return t_last_kernel; }

int rank_entries(int k1) { return k1 <= kDirectRankBits ? 1 << k1 : 256 + 9 * (1 << (k1 - 8)); }

int dp_lds_bytes(const StepShape &s, int amode, int n_rank, int teams) {
    int64_t bytes = 8LL * s.Wn * s.Bi;
    if (amode == kActiveLds) bytes += 8LL * s.Wa * s.Bi;
    bytes *= teams;
    const int64_t nt = s.p >= 2 ? s.Wq + n_rank : 0;
    bytes += 2LL * ((nt + 1) & ~1LL);
    StepShape s2 = s;
    s2.amode = amode;
    bytes += 4LL * split_lds_words(s2);
    bytes = (bytes + 15) & ~15LL;
    return bytes > (1 << 30) ? (1 << 30) : (int)bytes;
}

int chain_lds_bytes(int k1, int wmax, int bi, int tab_entries, int teams) {
    int64_t bytes = 8LL * bi * (k1 + 2LL * wmax) * teams + 2LL * tab_entries;
    bytes = (bytes + 15) & ~15LL;
    return bytes > (1 << 30) ? (1 << 30) : (int)bytes;
}

namespace {

template <bool WAVE, bool MOD, int TPB>
hipError_t chain_launch(const ChainArgs &c, int lds, hipStream_t st) {
    hipError_t e = allow_lds(dp_chain_kernel<WAVE, MOD, TPB>, lds);
    if (e != hipSuccess) return e;
    const int64_t teams = WAVE ? TPB / kWave : 1;
    const int64_t blocks =
        std::min<int64_t>((c.d.n * c.d.planes + teams - 1) / teams, 2 * resident_blocks(lds, TPB));
    name_kernel("dp_chain_kernel<%s, %s, %d>", tf(WAVE), tf(MOD), TPB);
    dp_chain_kernel<WAVE, MOD, TPB><<<dim3((unsigned)blocks), dim3(TPB), lds, st>>>(c);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dp_chain(const GraphBins &g, const ChainShape &cs, const uint8_t *col, const uint64_t *A,
                           const uint64_t *Npre, uint64_t *S, unsigned long long *flags, int wave_row_max,
                           hipStream_t st) {
    t_last_kernel[0] = 0;
    if (g.n <= 0) return hipSuccess;
    Modulus md;
    const int k1 = cs.k - 1;
    if (cs.steps < 2 || cs.steps > kMaxChainSteps || cs.a0 < 1 || cs.a0 + cs.steps > cs.k || cs.k > 16 ||
        cs.Bi < 1 || cs.Bi > kWave || (cs.Bi & (cs.Bi - 1)) || cs.B % cs.Bi || !S || !col ||
        (cs.a0 > 1) != (A != nullptr) || (g.n_split && !Npre) || !make_modulus(cs.mod, md))
        return hipErrorInvalidValue;
    ChainArgs c{};
    for (int i = 0; i < cs.steps; ++i) {
        const int a = cs.a0 + i;
        if ((a > 1 && !cs.split[i]) || cs.Wh[i] < 1 || cs.Wh[i] > cs.wmax || cs.nsplit[i] != a ||
            (i == 0 && a > 1 && cs.Wa[0] > cs.wmax))
            return hipErrorInvalidValue;
    }
    const int region = chain_lds_bytes(k1, cs.wmax, cs.Bi, 0);
    const bool wave = region <= wave_row_max && g.n * (cs.B / cs.Bi) >= kWaveRowsMin;
    const int teams = wave ? kWaves : 1;
    const int lds = chain_lds_bytes(k1, cs.wmax, cs.Bi, 0, teams);
    if (lds > kLdsPerCU) return hipErrorInvalidValue;
    const int tpb = !wave && lds > kWideLds ? kBlockWide : kBlock;
    DpArgs &a = c.d;
    a.rp = g.row_ptr; a.ci = g.col_idx; a.col = col; a.n = g.n;
    a.B = cs.B; a.Bi = cs.Bi; a.sh = log2_exact(cs.Bi); a.planes = cs.B / cs.Bi;
    a.p = 1; a.Wn = k1;
    a.Npre = const_cast<uint64_t *>(Npre);
    a.slot = g.n_split ? g.slot : nullptr; a.n_split = g.n_split;
    a.flags = flags;
    a.md = md;
    c.steps = cs.steps; c.a0 = cs.a0; c.wmax = cs.wmax; c.k1 = k1; c.Wa0 = cs.Wa[0];
    c.A = A; c.S = S;
    const int threads = tpb / teams;                 // threads building one row
    for (int i = 0; i < cs.steps; ++i) {
        ChainStepArgs &x = c.st[i];
        x.split = cs.split[i]; x.Wh = cs.Wh[i]; x.nsplit = cs.nsplit[i];
        // lanes per output entry: the power of two that shortens the longest chain
        x.eg = 1; x.lg_eg = 0;
        const int Ls = cs.Wh[i] * cs.Bi;
        int64_t best = -1;
        for (int lg = 0, G = 1; G <= kWave; ++lg, G *= 2) {
            if (G > 1 && G / 2 >= x.nsplit) break;
            const int64_t rounds = (Ls + (threads / G) - 1) / (threads / G);
            const int64_t chain = rounds * (((int64_t)x.nsplit + G - 1) / G + 2 * lg);
            if (best < 0 || chain < best) { best = chain; x.eg = G; x.lg_eg = lg; }
        }
    }
    if (wave) return cs.mod ? chain_launch<true, true, kBlock>(c, lds, st) : chain_launch<true, false, kBlock>(c, lds, st);
    if (tpb == kBlockWide)
        return cs.mod ? chain_launch<false, true, kBlockWide>(c, lds, st) : chain_launch<false, false, kBlockWide>(c, lds, st);
    return cs.mod ? chain_launch<false, true, kBlock>(c, lds, st) : chain_launch<false, false, kBlock>(c, lds, st);
}

int chain_wide_row_words(const ChainShape &cs, const int *limbs) {
    int w = 0;
    for (int i = 1; i + 1 < cs.steps; ++i) w = std::max(w, cs.Wh[i] * limbs[i]);
    return w;
}

int chain_wide_lds_bytes(int k1, int row_words, int bi, int teams) {
    int64_t bytes = 8LL * bi * (k1 + 2LL * row_words) * teams;
    bytes = (bytes + 15) & ~15LL;
    return bytes > (1 << 30) ? (1 << 30) : (int)bytes;
}

namespace {

template <bool WAVE, int TPB>
hipError_t chain_wide_launch(const ChainArgs &c, int lds, hipStream_t st) {
    hipError_t e = allow_lds(dp_chain_wide_kernel<WAVE, TPB>, lds);
    if (e != hipSuccess) return e;
    const int64_t teams = WAVE ? TPB / kWave : 1;
    const int64_t blocks =
        std::min<int64_t>((c.d.n * c.d.planes + teams - 1) / teams, 2 * resident_blocks(lds, TPB));
    name_kernel("dp_chain_wide_kernel<%s, %d>", tf(WAVE), TPB);
    dp_chain_wide_kernel<WAVE, TPB><<<dim3((unsigned)blocks), dim3(TPB), lds, st>>>(c);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dp_chain_wide(const GraphBins &g, const ChainShape &cs, const int *limbs, const uint8_t *col,
                                const uint64_t *Npre, uint64_t *S, unsigned long long *flags, int wave_row_max,
                                hipStream_t st) {
    t_last_kernel[0] = 0;
    if (g.n <= 0) return hipSuccess;
    const int k1 = cs.k - 1;
    if (!limbs || cs.a0 != 1 || cs.steps < 2 || cs.steps > kMaxChainSteps || cs.steps + 1 > cs.k || cs.k > 16 ||
        cs.Bi < 1 || cs.Bi > kWave || (cs.Bi & (cs.Bi - 1)) || cs.B % cs.Bi || !S || !col ||
        (g.n_split && !Npre) || cs.mod)
        return hipErrorInvalidValue;
    if (limbs[0] != 1) return hipErrorInvalidValue;           // the colour counts N'
    for (int i = 1; i < cs.steps; ++i)
        if (!cs.split[i] || cs.Wh[i] < 1 || cs.nsplit[i] != 1 + i || limbs[i] < limbs[i - 1] || limbs[i] > 4)
            return hipErrorInvalidValue;
    ChainArgs c{};
    const int wrow = chain_wide_row_words(cs, limbs);
    const int region = chain_wide_lds_bytes(k1, wrow, cs.Bi, 1);
    const bool wave = region <= wave_row_max && g.n * (cs.B / cs.Bi) >= kWaveRowsMin;
    const int teams = wave ? kWaves : 1;
    const int lds = chain_wide_lds_bytes(k1, wrow, cs.Bi, teams);
    if (lds > kLdsPerCU) return hipErrorInvalidValue;
    const int tpb = !wave && lds > kWideLds ? kBlockWide : kBlock;
    DpArgs &a = c.d;
    a.rp = g.row_ptr; a.ci = g.col_idx; a.col = col; a.n = g.n;
    a.B = cs.B; a.Bi = cs.Bi; a.sh = log2_exact(cs.Bi); a.planes = cs.B / cs.Bi;
    a.p = 1; a.Wn = k1;
    a.Npre = const_cast<uint64_t *>(Npre);
    a.slot = g.n_split ? g.slot : nullptr; a.n_split = g.n_split;
    a.flags = flags;
    c.steps = cs.steps; c.a0 = 1; c.wmax = wrow; c.k1 = k1; c.Wa0 = 1;
    c.S = S;
    const int threads = tpb / teams;
    for (int i = 0; i < cs.steps; ++i) {
        ChainStepArgs &x = c.st[i];
        x.split = cs.split[i]; x.Wh = cs.Wh[i]; x.nsplit = cs.nsplit[i];
        x.lin = i ? limbs[i - 1] : 1; x.lout = limbs[i];
        x.eg = 1; x.lg_eg = 0;
        const int Ls = cs.Wh[i] * cs.Bi;
        int64_t best = -1;
        for (int lg = 0, G = 1; G <= kWave; ++lg, G *= 2) {
            if (G > 1 && G / 2 >= x.nsplit) break;
            const int64_t rounds = (Ls + (threads / G) - 1) / (threads / G);
            const int64_t chain = rounds * (((int64_t)x.nsplit + G - 1) / G + 2 * lg);
            if (best < 0 || chain < best) { best = chain; x.eg = G; x.lg_eg = lg; }
        }
    }
    if (wave) return chain_wide_launch<true, kBlock>(c, lds, st);
    if (tpb == kBlockWide) return chain_wide_launch<false, kBlockWide>(c, lds, st);
    return chain_wide_launch<false, kBlock>(c, lds, st);
}

hipError_t launch_reduce_wide(int64_t n, const uint64_t *S, int W, int B, int Bi, int limbs,
                              unsigned long long *X, hipStream_t st) {
    t_last_kernel[0] = 0;
    if (n <= 0 || B <= 0) return hipSuccess;
    if (Bi < 1 || B % Bi || limbs < 1 || limbs > 4) return hipErrorInvalidValue;
    const int64_t total = n * W;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kBlock - 1) / kBlock, 1024));
    name_kernel("reduce_wide_kernel<%d>", limbs);
    if (limbs == 1) reduce_wide_kernel<1><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, X);
    else if (limbs == 2) reduce_wide_kernel<2><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, X);
    else if (limbs == 3) reduce_wide_kernel<3><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, X);
    else reduce_wide_kernel<4><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, X);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t *p, int64_t count, hipStream_t st) {
    t_last_kernel[0] = 0;
    if (count <= 0) return hipSuccess;
    name_kernel("zero_kernel");
    int64_t blocks = std::min<int64_t>((count + kBlock - 1) / kBlock, 8192);
    zero_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_color(const uint64_t *desc, int64_t n, int B, int k, const int32_t *perm,
                        uint8_t *col, hipStream_t st) {
    const int64_t total = n * B;
    t_last_kernel[0] = 0;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, kMaxStrideBlocks);
    name_kernel("color_kernel");
    color_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(desc, n, B, k, perm, col);
    return hipGetLastError();
}

bool root_step(const StepShape &s) {
    return s.a == 1 && s.p >= 2 && s.p == s.k - 1 && s.Wq == s.k - 1 && s.Wn == 1 && s.Wh == 1;
}

hipError_t launch_dp_split(const GraphBins &g, const StepShape &s, const StepTables &t,
                           const uint8_t *col, const uint64_t *P, uint64_t *Npre,
                           unsigned long long *flags, hipStream_t st) {
    t_last_kernel[0] = 0;
    if (g.n_split == 0 || g.n_split_items == 0 || root_step(s)) return hipSuccess;   // the root kernel sums every row
    if (!shape_ok(s) || (s.p >= 2 && (!P || !t.unrank || !t.rank))) return hipErrorInvalidValue;
    hipError_t e = launch_zero_u64(Npre, g.n_split * (int64_t)s.Wn * s.B, st);
    if (e != hipSuccess) return e;
    StepShape s1 = s;
    s1.amode = kActiveLeaf;                            // the pre-pass stages no active row or split table
    const DpArgs a = make_args(g, s1, t, col, P, nullptr, Npre, nullptr, flags, 1);
    const int lds = dp_lds_bytes(s1, kActiveLeaf, t.n_rank, 1);
    return s.mod ? split_dispatch<true>(s1, a, lds, st) : split_dispatch<false>(s1, a, lds, st);
}

hipError_t launch_dp_row(const GraphBins &g, const StepShape &s, const StepTables &t,
                         const uint8_t *col, const uint64_t *P, const uint64_t *A,
                         const uint64_t *Npre, uint64_t *S, unsigned long long *flags,
                         hipStream_t st) {
    t_last_kernel[0] = 0;
    if (g.n <= 0) return hipSuccess;
    if (!shape_ok(s) || !S || (s.p >= 2 && (!P || !t.unrank || !t.rank)) ||
        (s.amode != kActiveLeaf && (!A || !t.split)) || (g.n_split && !Npre))
        return hipErrorInvalidValue;
    if (root_step(s)) {
        // the root step of a template on all k colours reads one word per visit
        DpArgs a = make_args(g, s, t, col, P, nullptr, Npre, S, flags, kWaves);
        const int64_t blocks = std::min<int64_t>((a.n * a.planes + kWaves - 1) / kWaves, 2 * resident_blocks(0));
        name_kernel("dp_root_kernel<%s>", tf(s.mod != 0));
        if (s.mod) dp_root_kernel<true><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(a);
        else dp_root_kernel<false><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(a);
        return hipGetLastError();
    }
    // steps whose per-row LDS is small run one row per wavefront, when there
    // are enough rows to keep every wavefront slot of the chip busy (on a
    // small graph a row's latency matters more than the rows in flight)
    const int region = 8 * (s.Wn * s.Bi + (s.amode == kActiveLds ? s.Wa * s.Bi : 0));
    const bool wave = region <= s.wave_row_max && g.n * (s.B / s.Bi) >= kWaveRowsMin;
    const int teams = wave ? kWaves : 1;
    const int lds = dp_lds_bytes(s, s.amode, t.n_rank, teams);
    const DpArgs a = make_args(g, s, t, col, P, A, Npre, S, flags, teams, wide_workgroup(s, lds, wave) ? kBlockWide : kBlock);
    if (s.mod && wave) {
        if (s.amode == kActiveLeaf) return row_dispatch<kActiveLeaf, true, true>(s, a, lds, st);
        if (s.amode == kActiveLds) return row_dispatch<kActiveLds, true, true>(s, a, lds, st);
        return row_dispatch<kActiveGlobal, true, true>(s, a, lds, st);
    }
    if (s.mod) {
        if (s.amode == kActiveLeaf) return row_dispatch<kActiveLeaf, false, true>(s, a, lds, st);
        if (s.amode == kActiveLds) return row_dispatch<kActiveLds, false, true>(s, a, lds, st);
        return row_dispatch<kActiveGlobal, false, true>(s, a, lds, st);
    }
    if (wave) {
        if (s.amode == kActiveLeaf) return row_dispatch<kActiveLeaf, true, false>(s, a, lds, st);
        if (s.amode == kActiveLds) return row_dispatch<kActiveLds, true, false>(s, a, lds, st);
        return row_dispatch<kActiveGlobal, true, false>(s, a, lds, st);
    }
    if (s.amode == kActiveLeaf) return row_dispatch<kActiveLeaf, false, false>(s, a, lds, st);
    if (s.amode == kActiveLds) return row_dispatch<kActiveLds, false, false>(s, a, lds, st);
    return row_dispatch<kActiveGlobal, false, false>(s, a, lds, st);
}

hipError_t launch_reduce(int64_t n, const uint64_t *S, int W, int B, int Bi, uint64_t mod,
                         unsigned long long *X, unsigned long long *flags, hipStream_t st) {
    t_last_kernel[0] = 0;
    if (n <= 0 || B <= 0) return hipSuccess;
    Modulus md;
    if (Bi < 1 || B % Bi || !make_modulus(mod, md)) return hipErrorInvalidValue;
    const int64_t total = n * W;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kBlock - 1) / kBlock, 1024));
    name_kernel("reduce_kernel<%s>", tf(mod != 0));
    if (mod) reduce_kernel<true><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, md, X, flags);
    else reduce_kernel<false><<<dim3(blocks, (unsigned)B), dim3(kBlock), 0, st>>>(n, S, W, Bi, md, X, flags);
    return hipGetLastError();
}

int64_t valu_probe_threads() { return (int64_t)kCUs * 4 * 8 * kWave; }   // 8 wavefronts per SIMD

hipError_t launch_valu_probe(int form, uint64_t seed, int iters, unsigned long long *out, double *mul_adds,
                             hipStream_t st) {
    const unsigned blocks = (unsigned)(valu_probe_threads() / kBlock);
    *mul_adds = (double)valu_probe_threads() * iters * kProbeChains;
    name_kernel("valu_probe_kernel<%d>", form);
    if (form == 0) valu_probe_kernel<0><<<dim3(blocks), dim3(kBlock), 0, st>>>(seed, iters, out);
    else if (form == 1) valu_probe_kernel<1><<<dim3(blocks), dim3(kBlock), 0, st>>>(seed, iters, out);
    else if (form == 2) valu_probe_kernel<2><<<dim3(blocks), dim3(kBlock), 0, st>>>(seed, iters, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_hom_step(const GraphBins &g, const double *A, const double *P, double *S, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    if (!S) return hipErrorInvalidValue;
    const int64_t blocks = std::min<int64_t>((g.n + kWaves - 1) / kWaves, kMaxStrideBlocks);
    hom_step_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(g.n, g.row_ptr, g.col_idx, A, P, S);
    return hipGetLastError();
}

hipError_t launch_hom_sum(int64_t n, const double *S, double *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    hom_sum_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(n, S, out);
    return hipGetLastError();
}

hipError_t launch_hom_max(int64_t n, const double *S, double *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    hom_max_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(n, S, (unsigned long long *)out);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace sc
