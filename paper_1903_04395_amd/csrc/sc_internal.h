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

// How a step runs (see step_mode()).
enum StepMode {
    kStepFusedHist = 0,    // p = 1: colour histogram and multiply-add in one row kernel
    kStepFusedGather = 1,  // narrow passive rows: neighbour sum and multiply-add in one row kernel
    kStepStaged = 2,       // neighbour-sum table N, then the LDS row kernel
    kStepGlobal = 3        // neighbour-sum table N, then select / multiply-add from global memory
};

struct ExecOpts {
    bool fuse = true;          // allow the fused modes
    int fuse_max_cols = 512;   // widest passive row (Wp*B uint64) the fused gather takes
    int lds_max = 64 * 1024;   // LDS bytes a row kernel may use
};

// One DP step: attach the subtree of `child` (passive, size p) to what `node`
// has built so far (active, size a); h = a + p.  Buffers are indices into
// Plan::bufs; -1 means the implicit single-vertex table (computed from the
// colours on the fly) or, for buf_n, a neighbour sum that stays in LDS.
struct Step {
    int node, child;
    int h, a, p;
    int mode;
    int buf_a, buf_p, buf_n, buf_s;
    bool last;
};

struct Buf {
    int size;          // sub-template size (table has binom(k,size) colour-set columns)
    uint64_t bytes;    // n * binom(k,size) * batch * 8, rounded to 256
    uint64_t offset;   // byte offset inside the run arena
};

struct Plan {
    int t = 0, k = 0, root = 0, batch = 1;
    int64_t n = 0, nnz = 0;
    std::vector<int> child_ptr, child_idx, subtree;
    std::vector<Step> steps;
    std::vector<Buf> bufs;
    uint64_t arena_bytes = 0;
    double spmm_updates = 0, ema_updates = 0, lemma1_ops = 0, compulsory_bytes = 0, cost = 0;
    ExecOpts opts;
};

int step_mode(int k, int h, int a, int p, int batch, const ExecOpts &o);
int row_lds_need(int k, int a, int p, int batch, int mode);

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

// Split table of a step: for every output colour set I_s (in index order),
// binom(h,a) packed pairs (I_a | I_p << 16).
std::vector<uint32_t> split_table(int k, int h, int a);
// "Drop one colour" table for a = 1: entry [I_s * k + c] is the index of
// C_s \ {c} among (h-1)-sets, or -1 when c is not in C_s.
std::vector<int16_t> drop_table(int k, int h);

void fill_plan_info(const Plan &p, double aut, sc_plan_info_t *out);

}  // namespace sc
