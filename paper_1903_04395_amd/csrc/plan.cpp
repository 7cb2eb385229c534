// Host-side planning for the colour-coding DP: template checks, rooting and
// child order (Section 2.1, phase 2), the per-step sizes (h, a, p), Lemma 1
// operation counts, a static memory plan for the count tables, the Eq. 1
// colour-set index and the split / rank index tables the kernels read.
#include "sc_internal.h"
#include "kernels.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <limits>

namespace sc {

uint64_t binom(int n, int r) {
    if (r < 0 || n < 0 || r > n) return 0;
    static uint64_t pascal[65][65];
    static bool init = false;
    if (!init) {
        for (int i = 0; i <= 64; ++i) {
            pascal[i][0] = 1;
            for (int j = 1; j <= i; ++j)
                pascal[i][j] = pascal[i - 1][j - 1] + (j <= i - 1 ? pascal[i - 1][j] : 0);
        }
        init = true;
    }
    return pascal[n][r];
}

int64_t colorset_rank(uint32_t mask) {
    int64_t idx = 0;
    int i = 1;
    while (mask) {
        int c = __builtin_ctz(mask);
        idx += (int64_t)binom(c, i++);
        mask &= mask - 1;
    }
    return idx;
}

std::string check_tree(int t, const int32_t *edges) {
    if (t < 1 || t > SC_MAX_T) return "template size must be in [1, 16]";
    if (t > 1 && !edges) return "edges is NULL";
    std::vector<int> parent(t);
    for (int i = 0; i < t; ++i) parent[i] = i;
    std::function<int(int)> find = [&](int x) { return parent[x] == x ? x : parent[x] = find(parent[x]); };
    for (int e = 0; e < t - 1; ++e) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= t || v >= t) return "template edge endpoint out of range";
        if (u == v) return "template has a self-loop";
        int ru = find(u), rv = find(v);
        if (ru == rv) return "template edges contain a cycle (not a tree)";
        parent[ru] = rv;
    }
    return "";
}

void root_tree(int t, const int32_t *edges, int root, int order,
               std::vector<int> &child_ptr, std::vector<int> &child_idx) {
    std::vector<std::vector<int>> adj(t), kids(t);
    for (int e = 0; e < t - 1; ++e) {
        adj[edges[2 * e]].push_back(edges[2 * e + 1]);
        adj[edges[2 * e + 1]].push_back(edges[2 * e]);
    }
    std::vector<int> par(t, -1), bfs{root}, size(t, 1);
    std::vector<char> seen(t, 0);
    seen[root] = 1;
    for (size_t i = 0; i < bfs.size(); ++i)
        for (int w : adj[bfs[i]])
            if (!seen[w]) { seen[w] = 1; par[w] = bfs[i]; bfs.push_back(w); kids[bfs[i]].push_back(w); }
    for (int i = t - 1; i > 0; --i) size[par[bfs[i]]] += size[bfs[i]];
    child_ptr.assign(t + 1, 0);
    child_idx.clear();
    for (int u = 0; u < t; ++u) {
        auto &c = kids[u];
        std::stable_sort(c.begin(), c.end(), [&](int x, int y) {
            return order == 0 ? (size[x] < size[y] || (size[x] == size[y] && x < y))
                              : (size[x] > size[y] || (size[x] == size[y] && x < y));
        });
        for (int w : c) child_idx.push_back(w);
        child_ptr[u + 1] = (int)child_idx.size();
    }
}

int step_lds_bytes(int k, int a, int p, int bi, int amode) {
    kern::StepShape sh;
    sh.k = k; sh.a = a; sh.p = p; sh.B = bi; sh.Bi = bi;
    sh.Wq = p >= 2 ? (int)binom(k - 1, p - 1) : 0;
    sh.Wn = (int)binom(k - 1, p);
    sh.Wa = (int)binom(k - 1, a - 1);
    sh.Wh = (int)binom(k - 1, a + p - 1);
    sh.nsplit = (int)binom(a + p - 1, a - 1);
    sh.amode = amode;
    return kern::dp_lds_bytes(sh, amode, kern::rank_entries(k - 1));
}

void lemma1_counts(Plan &P, int64_t n) {
    const int k = P.k;
    const double nnz = (double)P.nnz;
    P.lemma1_ops = P.spmm_updates = P.ema_updates = 0;
    for (const Step &s : P.steps) {
        const double Wp = (double)binom(k, s.p), Wh = (double)binom(k, s.h);
        P.lemma1_ops += nnz * Wp + (double)n * Wh * (double)binom(s.h, s.p);
        P.spmm_updates += nnz * Wp;
        P.ema_updates += s.a > 1 ? (double)n * Wh * (double)binom(s.h, s.a) : (double)n * Wh;
    }
}

int chain_lds_bytes(int k, int wmax, int bi, int tab_entries) {
    return kern::chain_lds_bytes(k - 1, wmax, bi, tab_entries);
}

void chain_extent(int k, int a0, int steps, int &wmax, int &tab_entries) {
    wmax = a0 > 1 ? (int)binom(k - 1, a0 - 1) : 0;
    for (int i = 0; i < steps; ++i) wmax = std::max<int>(wmax, (int)binom(k - 1, a0 + i));   // step (a+1, a, 1)
    tab_entries = 0;            // the split tables are read through the caches
}

namespace {

// First-fit placement of buffers inside one arena, in allocation order.
struct Arena {
    std::vector<std::pair<uint64_t, uint64_t>> free_;   // (offset, length), sorted
    uint64_t end = 0;
    uint64_t alloc(uint64_t bytes) {
        for (size_t i = 0; i < free_.size(); ++i)
            if (free_[i].second >= bytes) {
                uint64_t off = free_[i].first;
                free_[i].first += bytes;
                free_[i].second -= bytes;
                if (free_[i].second == 0) free_.erase(free_.begin() + i);
                return off;
            }
        // extend, merging a free tail block
        if (!free_.empty() && free_.back().first + free_.back().second == end) {
            uint64_t off = free_.back().first;
            free_.pop_back();
            end = off + bytes;
            return off;
        }
        uint64_t off = end;
        end += bytes;
        return off;
    }
    void release(uint64_t off, uint64_t bytes) {
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (uint64_t)0));
        it = free_.insert(it, {off, bytes});
        size_t i = it - free_.begin();
        if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
            free_[i].second += free_[i + 1].second;
            free_.erase(free_.begin() + i + 1);
        }
        if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
            free_[i - 1].second += free_[i].second;
            free_.erase(free_.begin() + i);
        }
    }
};

uint64_t table_bytes(int64_t n, int k, int size, int batch) {
    uint64_t b = (uint64_t)n * binom(k - 1, size - 1) * (uint64_t)batch * 8;
    return (b + 255) & ~(uint64_t)255;
}

// Colourings interleaved per plane: the largest power of two dividing
// `batch`, at most `cap` (0: 64), with which every step's row kernel fits
// `lds_max` bytes of LDS (without a staged active row); 1 if none does.
int pick_interleave(const Plan &P, int cap, int lds_max) {
    int bi = 1;
    while (bi < 64 && P.batch % (2 * bi) == 0 && (cap == 0 || 2 * bi <= cap)) bi *= 2;
    for (; bi > 1; bi /= 2) {
        bool fits = true;
        for (const Step &s : P.steps)
            if (step_lds_bytes(P.k, s.a, s.p, bi, s.a > 1 ? kActGlobal : kActLeaf) > lds_max) fits = false;
        for (const Chain &ch : P.chains)
            if (chain_lds_bytes(P.k, ch.wmax, bi, ch.tab_entries) > lds_max) fits = false;
        if (fits) break;
    }
    return bi;
}

}  // namespace

bool build_plan(int t, int root, const std::vector<int> &child_ptr,
                const std::vector<int> &child_idx, int k, int64_t n, int64_t nnz,
                int batch, const ExecOpts &o, Plan &P, std::string &err) {
    P = Plan();
    P.t = t; P.k = k; P.root = root; P.n = n; P.nnz = nnz; P.batch = batch;
    P.child_ptr = child_ptr; P.child_idx = child_idx;
    P.opts = o;
    if (k < t || k > SC_MAX_K) { err = "need t <= k <= 16"; return false; }
    // subtree sizes and a check that the rooted tree spans 0..t-1 once
    P.subtree.assign(t, 0);
    std::vector<int> seen(t, 0);
    std::function<int(int)> sz = [&](int u) -> int {
        if (seen[u]++) return -(1 << 20);
        int s = 1;
        for (int e = child_ptr[u]; e < child_ptr[u + 1]; ++e) s += sz(child_idx[e]);
        return P.subtree[u] = s;
    };
    if ((int)child_ptr.size() != t + 1 || child_ptr[0] != 0 || child_ptr[t] != t - 1 ||
        root < 0 || root >= t) { err = "malformed plan"; return false; }
    for (int e = 0; e < t - 1; ++e)
        if (child_idx[e] < 0 || child_idx[e] >= t) { err = "malformed plan"; return false; }
    if (sz(root) != t) { err = "plan is not a rooted spanning tree"; return false; }
    for (int u = 0; u < t; ++u) if (seen[u] != 1) { err = "plan is not a rooted spanning tree"; return false; }

    Arena arena;
    // stored: a table in the arena; else a chain's intermediate (LDS only)
    auto new_buf = [&](int size, bool stored) {
        Buf b{size, table_bytes(n, k, size, batch), 0, stored};
        if (stored) b.offset = arena.alloc(b.bytes);
        P.bufs.push_back(b);
        return (int)P.bufs.size() - 1;
    };
    auto drop = [&](int id) {
        if (id >= 0 && P.bufs[id].stored) arena.release(P.bufs[id].offset, P.bufs[id].bytes);
    };
    // A run of two or more single-vertex children attached to the same vertex
    // one after another becomes one chain kernel when its two widest rows and
    // its index tables fit the LDS limit with one colouring per plane.
    auto chain_fuse = [&](int u) {
        const int c0 = child_ptr[u], c1 = child_ptr[u + 1];
        std::vector<char> fuse(c1 - c0, 0);
        if (!o.chain) return fuse;
        int size = 1;
        for (int e = c0; e < c1;) {
            if (P.subtree[child_idx[e]] != 1) { size += P.subtree[child_idx[e]]; ++e; continue; }
            int r = e;
            while (r < c1 && P.subtree[child_idx[r]] == 1) ++r;
            int wmax = 0, tab = 0;
            chain_extent(k, size, r - e, wmax, tab);
            if (r - e >= 2 && chain_lds_bytes(k, wmax, 1, tab) <= o.lds_max)
                for (int j = e; j + 1 < r; ++j) fuse[j - c0] = 1;
            size += r - e;
            e = r;
        }
        return fuse;
    };

    // post-order walk: the subtree of u is built by attaching its children in order
    std::function<int(int)> walk = [&](int u) -> int {
        int cur = -1, size = 1;
        const std::vector<char> fuse = chain_fuse(u);
        for (int e = child_ptr[u]; e < child_ptr[u + 1]; ++e) {
            int w = child_idx[e];
            int pb = walk(w);
            Step s;
            s.node = u; s.child = w;
            s.a = size; s.p = P.subtree[w]; s.h = s.a + s.p;
            s.buf_a = cur; s.buf_p = pb;
            s.mode = s.p == 1 ? kStepHist : kStepGather;
            s.amode = kActLeaf;
            s.lds_bytes = 0;
            s.fuse_next = fuse[e - child_ptr[u]] != 0;
            s.buf_s = new_buf(s.h, !s.fuse_next);
            s.last = false;
            drop(s.buf_a);
            drop(s.buf_p);
            P.steps.push_back(s);
            cur = s.buf_s;
            size = s.h;
        }
        return cur;
    };
    int top = walk(root);
    if (!P.steps.empty()) P.steps.back().last = true;
    (void)top;
    P.arena_bytes = arena.end;
    for (int i = 0; i < (int)P.steps.size(); ++i) {
        if (!P.steps[i].fuse_next || (i > 0 && P.steps[i - 1].fuse_next)) continue;
        Chain ch{i, i, 0, 0};
        while (P.steps[ch.last].fuse_next) ++ch.last;
        chain_extent(k, P.steps[i].a, ch.last - i + 1, ch.wmax, ch.tab_entries);
        P.chains.push_back(ch);
    }

    // Interleave and per-step LDS use.  A row kernel needs at least the
    // neighbour-sum row of one colouring and the index tables; when even that
    // exceeds lds_max (k = 16) the kernel takes what it needs, up to 160 KB.
    P.interleave = pick_interleave(P, o.interleave, o.lds_max);
    for (Step &s : P.steps) {
        const int base = step_lds_bytes(k, s.a, s.p, P.interleave, s.a > 1 ? kActGlobal : kActLeaf);
        if (base > 160 * 1024) { err = "a step's neighbour-sum row does not fit in LDS"; return false; }
        // The active row is staged in LDS when it fits the limit and its
        // entries are read more than once: an active set C1 pairs with
        // binom(k - a, p) output sets (one when the step's output is the whole
        // colour set, where staging only costs occupancy).  Other rows are
        // read from global memory, where the row stays in the caches.
        s.amode = kActLeaf;
        if (s.a > 1) {
            const int staged = step_lds_bytes(k, s.a, s.p, P.interleave, kActLds);
            const bool reused = binom(k - s.a, s.p) > 1;
            s.amode = reused && staged <= std::max(o.lds_max, base) ? kActLds : kActGlobal;
        }
        s.lds_bytes = step_lds_bytes(k, s.a, s.p, P.interleave, s.amode);
    }

    // Per colouring: Lemma 1 counts of the paper's layout (the benchmark's
    // update counts), the updates executed in the rooted-colour layout, and a
    // byte model of that layout.
    lemma1_counts(P, n);
    for (const Step &s : P.steps) {
        const double Rq = (double)binom(k - 1, s.p - 1), Rn = (double)binom(k - 1, s.p);
        const double Ra = (double)binom(k - 1, s.a - 1), Rh = (double)binom(k - 1, s.h - 1);
        const double madds = s.a > 1 ? (double)n * Rh * (double)binom(s.h - 1, s.a - 1) : (double)n * Rn;
        P.exec_updates += (s.p > 1 ? (double)nnz * Rq : (double)nnz) + madds;
        double bytes = 8.0 * n * ((s.a > 1 ? Ra : 0) + (s.p > 1 ? Rq : 0) + Rh);
        bytes += (double)n;                                        // colours
        bytes += 4.0 * nnz + 8.0 * (n + 1);                        // adjacency
        P.compulsory_bytes += bytes;
        // gathered rows miss the caches almost always; a colour read per
        // neighbour costs about a 16-byte sector; a u64 multiply-add is
        // about half a byte's time at the HBM rate
        const double gather = s.p >= 2 ? 8.0 * nnz * Rq : 16.0 * nnz;
        P.cost += bytes + gather + 0.5 * madds;
    }
    return true;
}

bool choose_plan(int t, const int32_t *edges, int root, int k, int64_t n, int64_t nnz,
                 int batch, const ExecOpts &o, Plan &out, std::string &err) {
    std::string m = check_tree(t, edges);
    if (!m.empty()) { err = m; return false; }
    if (root >= t) { err = "root out of range"; return false; }
    // The rooted tree is chosen on the cost of one colouring, so the same
    // template gets the same plan (and the same overflow flags) at any batch.
    bool found = false;
    double best_cost = 0;
    uint64_t best_arena = 0;
    std::vector<int> best_cp, best_ci;
    int best_root = 0;
    for (int r = (root < 0 ? 0 : root); r < (root < 0 ? t : root + 1); ++r)
        for (int order = 0; order < 2; ++order) {
            std::vector<int> cp, ci;
            root_tree(t, edges, r, order, cp, ci);
            Plan p;
            if (!build_plan(t, r, cp, ci, k, n, nnz, 1, o, p, err)) return false;
            if (!found || p.cost < best_cost || (p.cost == best_cost && p.arena_bytes < best_arena)) {
                best_cost = p.cost;
                best_arena = p.arena_bytes;
                best_cp = cp;
                best_ci = ci;
                best_root = r;
                found = true;
            }
        }
    if (!found) return false;
    return build_plan(t, best_root, best_cp, best_ci, k, n, nnz, batch, o, out, err);
}

// Automorphisms of an unrooted tree: root it at its centre (or cut the central
// edge), then aut(u) = prod aut(children) * prod (multiplicity of each
// isomorphism class of child subtrees)!.  Isomorphism classes of rooted
// subtrees get integer labels from the sorted labels of their children.
double tree_automorphisms(int t, const std::vector<std::pair<int,int>> &edges) {
    if (t <= 1) return 1.0;
    std::vector<std::vector<int>> adj(t);
    for (auto &e : edges) { adj[e.first].push_back(e.second); adj[e.second].push_back(e.first); }
    // centre(s) by repeatedly stripping leaves
    std::vector<int> deg(t), layer, removed(t, 0);
    for (int u = 0; u < t; ++u) { deg[u] = (int)adj[u].size(); if (deg[u] <= 1) layer.push_back(u); }
    int left = t;
    while (left > 2) {
        std::vector<int> next;
        for (int u : layer) {
            removed[u] = 1; --left;
            for (int w : adj[u]) if (!removed[w] && --deg[w] == 1) next.push_back(w);
        }
        layer = next;
    }
    std::vector<int> centres;
    for (int u = 0; u < t; ++u) if (!removed[u]) centres.push_back(u);
    std::map<std::vector<int>, int> labels;
    std::function<std::pair<int, double>(int, int)> rooted = [&](int u, int par) {
        std::vector<int> kid_labels;
        double a = 1.0;
        for (int w : adj[u]) if (w != par) {
            auto r = rooted(w, u);
            kid_labels.push_back(r.first);
            a *= r.second;
        }
        std::sort(kid_labels.begin(), kid_labels.end());
        for (size_t i = 0; i < kid_labels.size();) {
            size_t j = i;
            while (j < kid_labels.size() && kid_labels[j] == kid_labels[i]) ++j;
            for (size_t m = 2; m <= j - i; ++m) a *= (double)m;
            i = j;
        }
        auto it = labels.find(kid_labels);
        int lab = it == labels.end() ? (labels[kid_labels] = (int)labels.size()) : it->second;
        return std::make_pair(lab, a);
    };
    if (centres.size() == 1) return rooted(centres[0], -1).second;
    auto x = rooted(centres[0], centres[1]);
    auto y = rooted(centres[1], centres[0]);
    return x.second * y.second * (x.first == y.first ? 2.0 : 1.0);
}

std::vector<uint32_t> split_table(int k, int h, int a) {
    const int per = (int)binom(h, a);
    const uint64_t sets = binom(k, h);
    std::vector<uint32_t> out(sets * (uint64_t)per);
    for (uint32_t ms = 0; ms < (1u << k); ++ms) {
        if (__builtin_popcount(ms) != h) continue;
        int64_t is = colorset_rank(ms);
        int q = 0;
        // subsets of ms with a elements, walking the submasks
        for (uint32_t ma = ms;; ma = (ma - 1) & ms) {
            if (__builtin_popcount(ma) == a) {
                uint32_t ia = (uint32_t)colorset_rank(ma), ip = (uint32_t)colorset_rank(ms ^ ma);
                out[(uint64_t)q++ * sets + is] = ia | (ip << 16);
            }
            if (!ma) break;
        }
    }
    return out;
}

std::vector<uint16_t> unrank_table(int k1, int sz) {
    std::vector<uint16_t> out(binom(k1, sz));
    for (uint32_t m = 0; m < (1u << k1); ++m)
        if (__builtin_popcount(m) == sz) out[colorset_rank(m)] = (uint16_t)m;
    return out;
}

std::vector<uint16_t> rank_table(int k1) {
    std::vector<uint16_t> out(kern::rank_entries(k1), 0);
    if (k1 <= kern::kDirectRankBits) {
        for (uint32_t m = 0; m < (1u << k1); ++m) out[m] = (uint16_t)colorset_rank(m);
        return out;
    }
    for (uint32_t lo = 0; lo < 256; ++lo) out[lo] = (uint16_t)colorset_rank(lo);
    // high part: colour 8 + c at order m + (its order among the high colours)
    for (uint32_t hi = 0; hi < (1u << (k1 - 8)); ++hi)
        for (int m = 0; m <= 8; ++m) {
            uint64_t idx = 0;
            int order = m;
            for (int c = 0; c < k1 - 8; ++c)
                if (hi & (1u << c)) idx += binom(8 + c, ++order);
            out[256 + hi * 9 + m] = (uint16_t)idx;
        }
    return out;
}

void fill_plan_info(const Plan &p, double aut, sc_plan_info_t *o) {
    std::memset(o, 0, sizeof(*o));
    o->t = p.t; o->k = p.k; o->root = p.root; o->n_steps = (int)p.steps.size();
    for (int i = 0; i <= p.t && i < (int)p.child_ptr.size(); ++i) o->child_ptr[i] = p.child_ptr[i];
    for (int i = 0; i < p.t - 1; ++i) o->child_idx[i] = p.child_idx[i];
    for (size_t i = 0; i < p.steps.size(); ++i) {
        o->step_h[i] = p.steps[i].h; o->step_a[i] = p.steps[i].a; o->step_p[i] = p.steps[i].p;
    }
    o->batch = p.batch;
    o->arena_bytes = p.arena_bytes;
    o->spmm_updates = p.spmm_updates;
    o->ema_updates = p.ema_updates;
    o->lemma1_ops = p.lemma1_ops;
    o->exec_updates = p.exec_updates;
    o->interleave = p.interleave;
    for (size_t i = 0; i < p.steps.size(); ++i) o->step_mode[i] = p.steps[i].mode;
    o->compulsory_bytes = p.compulsory_bytes;
    o->automorphisms = aut;
}

}  // namespace sc
