// Launchers for the gfx950 kernels of libsc (definitions in kernels.hip).
// Table layout everywhere: a table for sub-template size s in a pass of B
// colourings is uint64[n][binom(k,s) * B]; entry (v, colour set I, colouring r)
// lives at v * binom(k,s) * B + I * B + r.  Colours are uint8[n][B].
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sc {
namespace kern {

// Rows are binned by degree once per graph:
//  light rows  (deg <= kLightMax): one wavefront per row;
//  wide items  (deg >  kLightMax): one workgroup per (row, segment of `seg`
//              neighbours); rows with deg > seg are split into several
//              segments whose partial sums meet in global atomics.
constexpr int kLightMax = 64;

struct GraphBins {
    int64_t n = 0, nnz = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const int32_t *light_rows = nullptr;  int64_t n_light = 0;
    const int2 *wide_items = nullptr;     int64_t n_wide = 0;   // (row, segment)
    const int32_t *split_rows = nullptr;  int64_t n_split = 0;  // rows with deg > seg
    int seg = 0;
};

// col[v*B + r] = colour of vertex v in colouring first+r (SplitMix64 rule).
hipError_t launch_color(uint64_t seed, uint64_t first, int64_t n, int B, int k, uint8_t *col,
                        hipStream_t st);

// N = A * P for a table with L = W*B uint64 columns per row.
hipError_t launch_spmm(const GraphBins &g, const uint64_t *P, uint64_t *N, int64_t L, int B,
                       int chunk_cols, unsigned long long *flags, hipStream_t st);

// p = 1: N[v][c*B + r] = #{j in adj(v) : col[j*B + r] == c}, c < k.
hipError_t launch_hist(const GraphBins &g, const uint8_t *col, uint64_t *N, int B, int k,
                       hipStream_t st);

// a = 1: S[v][I*B + r] = N[v][drop[I*k + c]*B + r] if c = col[v*B+r] is in set I, else 0.
hipError_t launch_select(int64_t n, const uint8_t *col, const uint64_t *N, uint64_t *S, int B,
                         int k, int Wh, int Wp, const int16_t *drop, hipStream_t st);

// a >= 2: S[v][I*B + r] = sum over the nsplit pairs (Ia, Ip) of set I of
// A[v][Ia*B + r] * N[v][Ip*B + r].
hipError_t launch_ema(int64_t n, const uint64_t *A, const uint64_t *N, uint64_t *S, int B,
                      int Wa, int Wp, int Wh, int nsplit, const uint32_t *split,
                      unsigned long long *flags, hipStream_t st);

// Fused p >= 1 neighbour sum + multiply-add for one step (the neighbour-sum row
// never leaves LDS).  a == 1 uses `drop`, a >= 2 uses `split` and A.
hipError_t launch_fused(const GraphBins &g, const uint8_t *col, const uint64_t *P,
                        const uint64_t *A, uint64_t *S, int B, int k, int a, int p, int Wa,
                        int Wp, int Wh, int nsplit, const uint32_t *split, const int16_t *drop,
                        unsigned long long *flags, hipStream_t st);

// X[r] = sum_v sum_I S[v][I*B + r] (with carry flags); X must be zeroed first.
hipError_t launch_reduce(int64_t n, const uint64_t *S, int W, int B, unsigned long long *X,
                         unsigned long long *flags, hipStream_t st);

hipError_t launch_zero_u64(uint64_t *p, int64_t count, hipStream_t st);

}  // namespace kern
}  // namespace sc
