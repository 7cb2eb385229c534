// Launchers for the gfx950 kernels of libsc (definitions in kernels.hip).
//
// Rooted-colour table layout.  In colouring r, the table of a sub-template of
// size s is zero at M_s[v][C] unless C holds col_r(v) (the sub-template's root
// maps to v), so a row keeps only the colour sets that hold the row's own
// colour: W(s) = binom(k-1, s-1) entries per colouring.  Entry j of row v is
// the set {col_r(v)} + D_j, where D_j is the j-th (s-1)-subset, in Eq. 1 order,
// of the k-1 other colours renumbered 0..k-2 (colour x > col_r(v) becomes
// x - 1).  Single-vertex tables are all ones and never stored.
//
// A pass of B colourings keeps them as `planes` planes of Bi interleaved
// colourings (B = planes * Bi, Bi a power of two): entry (v, j, r) with
// r = plane * Bi + ri lives at ((plane * n + v) * W + j) * Bi + ri.
// Colours are uint8[n][B].
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sc {
namespace kern {

// Rows with more than `seg` neighbours ("split rows") have their neighbour
// sums built by a pre-pass over (row, segment) items whose partial sums meet
// in global atomics; every other row is summed inside the row kernel.
struct GraphBins {
    int64_t n = 0, nnz = 0;   // n: rows the tables hold (isolated vertices dropped when relabelled)
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const int32_t *split_rows = nullptr;  int64_t n_split = 0;        // rows with deg > seg
    const int2 *split_items = nullptr;    int64_t n_split_items = 0;  // (row, segment)
    const int32_t *slot = nullptr;        // [n]: index of a split row in split_rows, else -1
    int seg = 0;
};

// How a step reads its active table: a = 1 (the all-ones single-vertex table,
// so the step's output is the neighbour sum itself), staged in LDS, or read
// from global memory (rows too wide to stage).
enum ActiveMode { kActiveLeaf = 0, kActiveLds = 1, kActiveGlobal = 2 };

// Shape of one DP step in the rooted-colour layout (h = a + p).
struct StepShape {
    int k = 0, a = 0, p = 0;
    int B = 1, Bi = 1;                 // colourings per pass; interleaved per plane
    int Wq = 0;                        // binom(k-1, p-1): passive row entries
    int Wn = 0;                        // binom(k-1, p):   neighbour-sum entries
    int Wa = 0;                        // binom(k-1, a-1): active row entries
    int Wh = 0;                        // binom(k-1, h-1): output row entries
    int nsplit = 0;                    // binom(h-1, a-1): split pairs per output entry
    int amode = kActiveLeaf;
    int wave_row_max = 8192;           // per-row LDS bytes up to which each wavefront
                                       // builds a row of its own (0: never)
    uint64_t mod = 0;                  // 0: exact uint64 entries with carry flags; else the
                                       // entries are residues mod this prime (mod_supported)
};

// Host-built index tables of a step (device pointers).
struct StepTables {
    const uint32_t *split = nullptr;   // a >= 2: per output set, nsplit pairs (Ia | Ip << 16)
                                       // of the (k-1, h-1, a-1) split table
    const uint16_t *unrank = nullptr;  // p >= 2: masks of the (p-1)-subsets of k-1 colours
    const uint16_t *rank = nullptr;    // Eq. 1 rank of a mask of k-1 colours (see rank_entries)
    int n_rank = 0;                    // entries of `rank`
};

// Rank table of masks of k1 colours: for k1 <= kDirectRankBits the rank of
// every mask, R[m]; above, two lookups, rank(m) = R[m & 255] +
// R[256 + (m >> 8) * 9 + popcount(m & 255)].  rank_entries() is its length.
constexpr int kDirectRankBits = 12;
int rank_entries(int k1);

// Dynamic LDS bytes of the row and split kernels of a step whose rows are
// built by `teams` teams per workgroup (1: the workgroup; 4: one per wavefront).
int dp_lds_bytes(const StepShape &s, int amode, int n_rank, int teams = 1);

// A run of steps executed by one kernel: the first step (h0, a0, 1) attaches
// a single vertex to the active table (the all-ones single-vertex table when
// a0 = 1), and every later step attaches one more single vertex to the
// previous step's output.  Each step's neighbour sum is the row's neighbour
// colour counts, so a row needs them once; the intermediate outputs stay in
// LDS and only the last step's output is written.
constexpr int kMaxChainSteps = 16;
struct ChainShape {
    int k = 0, a0 = 1, steps = 0;      // colours; active size of the first step; steps
    int B = 1, Bi = 1;
    int wmax = 0;                      // widest row held in LDS (entries per colouring)
    // per step: active and output row entries, split pairs per output entry
    // (a = h - 1), and (a >= 2) its (k-1, h-1, a-1) split table
    int Wa[kMaxChainSteps] = {}, Wh[kMaxChainSteps] = {}, nsplit[kMaxChainSteps] = {};
    const uint32_t *split[kMaxChainSteps] = {};
    uint64_t mod = 0;
};
// Dynamic LDS bytes of a chain kernel: per team the neighbour colour counts
// and two rows of `wmax` entries per interleaved colouring, then `tab_entries`
// uint16 index-table entries shared by the workgroup.
int chain_lds_bytes(int k1, int wmax, int bi, int tab_entries, int teams = 1);
// Runs the chain over every row: A is the first step's active table (NULL for
// a0 = 1), S the last step's output; rows above the segment size take their
// colour counts from Npre, written by launch_dp_split for the first step.
hipError_t launch_dp_chain(const GraphBins &g, const ChainShape &c, const uint8_t *col, const uint64_t *A,
                           const uint64_t *Npre, uint64_t *S, unsigned long long *flags, int wave_row_max,
                           hipStream_t st);

// Exact counts of a template that is one chain from a single vertex (the
// star rooted at its centre; a0 = 1), step i's entries kept as limbs[i]
// (1..4, limbs[0] = 1, non-decreasing) little-endian 64-bit limbs: the
// chain's last output to S (entry (v, j, r) limb l at
// (((plane*n + v)*W + j)*Bi + ri)*L + l, L the last step's limbs); a carry out
// of a step's top limb sets the colouring's flag.  chain_wide_row_words is
// the widest intermediate row (entries times limbs) per colouring, which
// chain_wide_lds_bytes takes.  launch_reduce_wide adds colouring r's n*W
// entries of `limbs` limbs into X[r][0..limbs] (limbs + 1 words, which must
// start at zero).
int chain_wide_row_words(const ChainShape &cs, const int *limbs);
int chain_wide_lds_bytes(int k1, int row_words, int bi, int teams = 1);
hipError_t launch_dp_chain_wide(const GraphBins &g, const ChainShape &c, const int *limbs, const uint8_t *col,
                                const uint64_t *Npre, uint64_t *S, unsigned long long *flags, int wave_row_max,
                                hipStream_t st);
hipError_t launch_reduce_wide(int64_t n, const uint64_t *S, int W, int B, int Bi, int limbs,
                              unsigned long long *X, hipStream_t st);

// col[v*B + r] = colour of vertex v in colouring first+r (SplitMix64 rule),
// drawn from the original id perm[v] when the graph was relabelled (perm != NULL);
// desc[0] = seed and desc[1] = first live in device memory.
hipError_t launch_color(const uint64_t *desc, int64_t n, int B, int k, const int32_t *perm,
                        uint8_t *col, hipStream_t st);

// Whether s is the root step (k, 1, k-1) of a template on all k colours: its
// neighbour sum is one entry, which the row kernel sums for every row (split
// rows included), so the step has no pre-pass.
bool root_step(const StepShape &s);

// Neighbour sums of the split rows into Npre[planes][n_split][Wn * Bi]
// (zeroed here first), from the passive table P (p >= 2) or the colours (p = 1).
hipError_t launch_dp_split(const GraphBins &g, const StepShape &s, const StepTables &t,
                           const uint8_t *col, const uint64_t *P, uint64_t *Npre,
                           unsigned long long *flags, hipStream_t st);

// One DP step: for every row v and plane, the neighbour sum N'[v] (the sets
// without col_r(v)) is built in LDS -- scattered from the neighbours' passive
// rows (p >= 2), counted from their colours (p = 1), or copied from Npre for
// split rows -- and S[v] = sum over splits of A[v][Ia] * N'[v][Ip] is written
// (S[v] = N'[v] when a = 1).  The root step (k, 1, k-1) of a template on all
// k colours, whose neighbour sum is a single entry, reads one word of each
// neighbour's row instead (dp_root_kernel).
hipError_t launch_dp_row(const GraphBins &g, const StepShape &s, const StepTables &t,
                         const uint8_t *col, const uint64_t *P, const uint64_t *A,
                         const uint64_t *Npre, uint64_t *S, unsigned long long *flags,
                         hipStream_t st);

// X[r] = sum over rows and the W entries of colouring r of table S (with carry
// flags); X must be zeroed first.  mod != 0: S holds residues and X[r] ends
// congruent to the sum mod `mod` (not reduced; no flags).
hipError_t launch_reduce(int64_t n, const uint64_t *S, int W, int B, int Bi, uint64_t mod,
                         unsigned long long *X, unsigned long long *flags, hipStream_t st);

// Residue passes accept primes p = 2^w - c with 61 <= w <= 63 and odd c <= 2^16.
bool mod_supported(uint64_t p);

// Homomorphism counts (double): S[v] = A[v] * sum over the neighbours u of v
// of P[u], with A or P NULL standing for the single-vertex sub-template (all
// ones).  launch_hom_sum adds the sum of S[0..n) into *out.
hipError_t launch_hom_step(const GraphBins &g, const double *A, const double *P, double *S, hipStream_t st);
hipError_t launch_hom_sum(int64_t n, const double *S, double *out, hipStream_t st);
// *out = max(*out, the largest of S[0..n)) (S >= 0; *out must start at a value >= 0).
hipError_t launch_hom_max(int64_t n, const double *S, double *out, hipStream_t st);

hipError_t launch_zero_u64(uint64_t *p, int64_t count, hipStream_t st);

// Vector-ALU roof of the exact multiply-add (form 0: 128-bit product, 1: three
// 32-bit multiplies, 2: 32-bit second operand): a register-only loop of
// `iters` multiply-adds per chain; `out` holds valu_probe_threads() words;
// *mul_adds is set to the multiply-adds the launch performs.
int64_t valu_probe_threads();
hipError_t launch_valu_probe(int form, uint64_t seed, int iters, unsigned long long *out, double *mul_adds,
                             hipStream_t st);

// Name of the kernel instantiation the calling thread's last launcher call
// enqueued (as profilers print it, e.g. "dp_row_kernel<16, 1, false, 0, true,
// false, 256>"), or "" if that call launched nothing.
const char *last_kernel_name();

// Baselines for the pruning ablation (ablation.hip): one DP step of one
// colouring with tables in the paper's layout ([n][binom(k, s)], column =
// Eq. 1 rank), either FASCIA's (the passive column summed over the neighbours
// once per split) or PFASCIA's (neighbour sums N[n][binom(k, p)] once, then
// the split multiply-add).  A / P NULL: single-vertex child (from `col`, one
// colour per row).  split: (k, h, a) split table; pmask: masks of the
// p-subsets of k colours.  Overflow sets bit 0 of *flag.
enum { kAblFascia = 1, kAblPfascia = 2 };
hipError_t launch_ablation_step(int variant, const GraphBins &g, int k, int a, int p, const uint8_t *col,
                                const uint32_t *split, const uint16_t *pmask, const uint64_t *A,
                                const uint64_t *P, uint64_t *N, uint64_t *S, unsigned long long *flag,
                                hipStream_t st);

}  // namespace kern
}  // namespace sc
