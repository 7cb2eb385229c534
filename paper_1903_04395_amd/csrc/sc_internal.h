// Internal declarations shared by the host planner, runtime and kernel
// launchers of libsc.  Not part of the public ABI (that is include/sc.h).
#pragma once

#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>
#include <map>

#include "../../include/sc.h"

namespace sc {

// binom(n, r) for 0 <= n <= 64 (0 outside the triangle).
uint64_t binom(int n, int r);

// Eq. 1 (Section 3): index of a colour set given as a bitmask,
// I = sum_i binom(c_i, i) over its colours c_1 < c_2 < ... (i from 1).
int64_t colorset_rank(uint32_t mask);

// How a step builds its neighbour sum (both run as one fused row kernel).
enum StepMode {
    kStepHist = 0,     // p = 1: counts of the neighbours' colours
    kStepGather = 1    // p >= 2: scatter of the neighbours' passive rows
};

// How a step reads its active table (same values as kern::ActiveMode).
enum ActiveMode { kActLeaf = 0, kActLds = 1, kActGlobal = 2 };

struct ExecOpts {
    int interleave = 0;        // cap on colourings interleaved per plane (0: no cap)
    int lds_max = 64 * 1024;   // LDS bytes a row kernel may use
    int wave_row_max = 8192;   // per-row LDS bytes up to which a wavefront builds a row alone
    int chain = 1;             // runs of single-vertex attaches fused into one kernel
    int seg = 0;               // neighbours per work item of split rows (0: the context's segment size)
};

// One DP step: attach the subtree of `child` (passive, size p) to what `node`
// has built so far (active, size a); h = a + p.  Buffers are indices into
// Plan::bufs; -1 means the implicit single-vertex table (all ones in the
// rooted-colour layout).
struct Step {
    int node, child;
    int h, a, p;
    int mode;          // StepMode
    int amode;         // ActiveMode
    int lds_bytes;     // dynamic LDS of its row kernel
    int buf_a, buf_p, buf_s;
    bool last;
    // The next step attaches a single vertex to this step's output, and both
    // run in one chain kernel: this output lives only in that kernel's LDS.
    bool fuse_next;
};

struct Buf {
    int size;          // sub-template size (binom(k-1,size-1) entries per row and colouring)
    uint64_t bytes;    // n * binom(k-1,size-1) * batch * 8, rounded to 256
    uint64_t offset;   // byte offset inside the run arena
    bool stored;       // false: a chain's intermediate, never placed in the arena
};

// A run of steps [first, last] executed by one kernel: every step after the
// first attaches a single vertex to the previous step's output.
struct Chain {
    int first, last;
    int wmax;          // widest row (entries per colouring) the chain holds in LDS
    int tab_entries;   // uint16 index-table entries it stages in LDS
};

struct Plan {
    int t = 0, k = 0, root = 0, batch = 1;
    int interleave = 1;         // colourings interleaved per plane (power of two dividing batch)
    int64_t n = 0, nnz = 0;
    std::vector<int> child_ptr, child_idx, subtree;
    std::vector<Step> steps;
    std::vector<Buf> bufs;
    std::vector<Chain> chains;
    uint64_t arena_bytes = 0;
    double spmm_updates = 0, ema_updates = 0, lemma1_ops = 0, exec_updates = 0;
    double compulsory_bytes = 0, cost = 0;
    ExecOpts opts;
};

// Dynamic LDS bytes of a step's row kernel with `bi` interleaved colourings.
int step_lds_bytes(int k, int a, int p, int bi, int amode);
// The paper's per-colouring counts (Lemma 1) of plan P on a graph of n
// vertices and P.nnz nonzeros: spmm_updates, ema_updates, lemma1_ops.
void lemma1_counts(Plan &P, int64_t n);

// Dynamic LDS bytes of a chain kernel whose widest row has `wmax` entries and
// whose index tables hold `tab_entries` uint16 entries.
int chain_lds_bytes(int k, int wmax, int bi, int tab_entries);
// Widest row and index-table entries of a chain of `steps` single-vertex
// attaches starting from an active child of size a0, over k colours.
void chain_extent(int k, int a0, int steps, int &wmax, int &tab_entries);

// Validates an edge list as a tree on t vertices; returns "" or a message.
std::string check_tree(int t, const int32_t *edges);

// Rooted, ordered tree from edges: children sorted by subtree size
// ascending (order=0) or descending (order=1).
void root_tree(int t, const int32_t *edges, int root, int order,
               std::vector<int> &child_ptr, std::vector<int> &child_idx);

// Builds steps, buffers and the static memory plan for a rooted ordered tree.
// Fused steps have no neighbour-sum buffer.
bool build_plan(int t, int root, const std::vector<int> &child_ptr,
                const std::vector<int> &child_idx, int k, int64_t n, int64_t nnz,
                int batch, const ExecOpts &o, Plan &out, std::string &err);

// Chooses the root and child order with the lowest modelled cost (root < 0),
// or orders the children of the given root.
bool choose_plan(int t, const int32_t *edges, int root, int k, int64_t n, int64_t nnz,
                 int batch, const ExecOpts &o, Plan &out, std::string &err);

// |Aut(T)| of the unrooted template tree.
double tree_automorphisms(int t, const std::vector<std::pair<int,int>> &edges);

// Split table over k colours: for every colour set I_s of size h (in index
// order), binom(h,a) packed pairs (I_a | I_p << 16), pair-major: pair j of
// set I_s at [j * binom(k,h) + I_s], so threads taking consecutive sets read
// consecutive words.  A rooted-colour step (h, a, p) uses the table of
// (k-1, h-1, a-1).
std::vector<uint32_t> split_table(int k, int h, int a);
// Masks of the s-subsets of k1 colours in Eq. 1 order.
std::vector<uint16_t> unrank_table(int k1, int s);
// Eq. 1 rank of any mask m of k1 colours, laid out as kern::rank_entries()
// describes (one lookup up to 12 colours, two above).
std::vector<uint16_t> rank_table(int k1);

void fill_plan_info(const Plan &p, double aut, sc_plan_info_t *out);

}  // namespace sc
