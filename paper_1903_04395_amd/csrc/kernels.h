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
//  light rows  (deg <= kLightMax): one wavefront per row (colour histogram);
//  wide items  (deg >  kLightMax): one workgroup per (row, segment of `seg`
//              neighbours) (colour histogram);
//  tasks       every row with deg <= seg, and every `seg`-neighbour segment of
//              the rows with more (neighbour sum);
// rows with deg > seg ("split rows") are summed over several segments whose
// partial sums meet in global atomics.
constexpr int kLightMax = 64;

struct GraphBins {
    int64_t n = 0, nnz = 0;   // n: rows the tables hold (isolated vertices dropped when relabelled)
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const int32_t *light_rows = nullptr;  int64_t n_light = 0;
    const int2 *wide_items = nullptr;     int64_t n_wide = 0;   // (row, segment), split rows first
    int64_t n_split_items = 0;                                  // items of split rows
    const int2 *tasks = nullptr;          int64_t n_tasks = 0;  // neighbour-sum tasks, split rows first
    int64_t n_split_tasks = 0;
    const int32_t *split_rows = nullptr;  int64_t n_split = 0;  // rows with deg > seg
    const int32_t *slot = nullptr;        // [n]: index of a split row in split_rows, else -1
    int seg = 0;
};

// col[v*B + r] = colour of vertex v in colouring first+r (SplitMix64 rule),
// drawn from the original id perm[v] when the graph was relabelled (perm != NULL);
// desc[0] = seed and desc[1] = first live in device memory.
hipError_t launch_color(const uint64_t *desc, int64_t n, int B, int k, const int32_t *perm,
                        uint8_t *col, hipStream_t st);

// N = A * P for a table with L = W*B uint64 columns per row (the split rows of
// N must be zeroed first, see launch_zero_split_rows), in column tiles
// of tile_cols = 8, 16, 32 (lane groups over several neighbours) or 64, 128,
// 256 (wavefront-wide row slices) uint64.
hipError_t launch_spmm(const GraphBins &g, const uint64_t *P, uint64_t *N, int64_t L, int B,
                       int tile_cols, unsigned long long *flags, hipStream_t st);

// Zeroes the split rows of N (compact: rows of Npre[n_split][L]) before the
// neighbour sums of their segments add into them.
hipError_t launch_zero_split_rows(const GraphBins &g, bool compact, uint64_t *N, int64_t L,
                                  hipStream_t st);

// Neighbour sums of the split rows only, into the compact Npre[n_split][L].
hipError_t launch_spmm_split(const GraphBins &g, const uint64_t *P, uint64_t *Npre, int64_t L,
                             int B, int tile_cols, unsigned long long *flags, hipStream_t st);

// p = 1: N[v][c*B + r] = #{j in adj(v) : col[j*B + r] == c}, c < k.
hipError_t launch_hist(const GraphBins &g, const uint8_t *col, uint64_t *N, int B, int k,
                       hipStream_t st);
// The same for the split rows only, into the compact Npre[n_split][k*B].
hipError_t launch_hist_split(const GraphBins &g, const uint8_t *col, uint64_t *Npre, int B, int k,
                             hipStream_t st);

// a = 1: S[v][I*B + r] = N[v][drop[I*k + c]*B + r] if c = col[v*B+r] is in set I, else 0.
hipError_t launch_select(int64_t n, const uint8_t *col, const uint64_t *N, uint64_t *S, int B,
                         int k, int Wh, int Wp, const int16_t *drop, hipStream_t st);

// a >= 2: S[v][I*B + r] = sum over the nsplit pairs (Ia, Ip) of set I of
// A[v][Ia*B + r] * N[v][Ip*B + r].
hipError_t launch_ema(int64_t n, const uint64_t *A, const uint64_t *N, uint64_t *S, int B,
                      int Wa, int Wp, int Wh, int nsplit, const uint32_t *split,
                      unsigned long long *flags, hipStream_t st);

// Row kernel: one workgroup per row, N[v] and A[v] staged in LDS, then the
// select (a = 1) or the split multiply-add (a >= 2).  Modes: the neighbour-sum
// row comes from N (`src`, staged), is summed from the passive table (`src`,
// fused; Wp*B <= 2048) or counted from colours (fused histogram, p = 1).
// Fused modes read split rows from Npre.
enum { kModeStaged = 0, kModeGather = 1, kModeHist = 2 };
int row_lds_bytes(int k, int a, int Wa, int Wp, int B, int mode);
hipError_t launch_row(int mode, const GraphBins &g, const uint8_t *col, const uint64_t *src,
                      const uint64_t *Npre, const uint64_t *A, uint64_t *S, int B, int k, int a,
                      int Wa, int Wp, int Wh, int nsplit, const uint32_t *split,
                      const int16_t *drop, unsigned long long *flags, hipStream_t st);

// X[r] = sum_v sum_I S[v][I*B + r] (with carry flags); X must be zeroed first.
hipError_t launch_reduce(int64_t n, const uint64_t *S, int W, int B, unsigned long long *X,
                         unsigned long long *flags, hipStream_t st);

hipError_t launch_zero_u64(uint64_t *p, int64_t count, hipStream_t st);

}  // namespace kern
}  // namespace sc
