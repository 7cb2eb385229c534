/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the colour-coding
 * tree-counting dynamic program of Chen et al., "A GraphBLAS Approach for
 * Subgraph Counting" (HPDC'19).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What is computed, per colouring (Section 2.1, the three phases of colour
 * coding; Section 4.1, Eq. 2):
 *
 *   col : V -> [0,k)              one colour per graph vertex
 *   leaf table   M[v][{c}] = [col(v) == c]                      (bottom case)
 *   for each sub-template T_s = T_a (+) T_p (active/passive children):
 *     N[v][C2]   = sum_{j in adj(v)} M_p[j][C2]                 (Eq. 2, the
 *                  neighbour sum taken once per passive colour set = A * M_p)
 *     M_s[v][C]  = sum_{C1 (+) C2 = C, |C1| = |T_a|} M_a[v][C1] * N[v][C2]
 *   X = sum_v sum_{|C| = t} M_root[v][C]
 *
 * Colour sets are indexed by Eq. 1 (the combinatorial number system):
 * I(C) = sum_{i=1..h} binom(c_i, i) for c_1 < ... < c_h.
 *
 * Arithmetic is uint64.  Readings where the paper is silent:
 *  - the neighbour sum has no self term (N = A * M_p, the adjacency of a simple
 *    graph has a zero diagonal);
 *  - overflow: the per-colouring flag is set iff some usable N entry, some
 *    product M_a*N, some M_s entry or X, evaluated exactly from the stored
 *    uint64 operands, is >= 2^64.  An N entry N[v][C2] is usable when col(v)
 *    is not in C2: M_a[v][C1] is zero unless C1 holds col(v) (the root of T_a
 *    maps to v), and C1, C2 are disjoint, so an N entry whose set holds col(v)
 *    only ever meets zero active entries and cannot reach the count.  Stored
 *    values are residues mod 2^64.  Because every term is non-negative,
 *    whether a sum overflows does not depend on the order of summation.
 *  - colours come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): colouring
 *    r of vertex v takes output number r*2^40 + v of the generator seeded with
 *    `seed`, mapped to [0,k) by a 64x64 multiply-high.
 *
 * The plan (root and the order in which each vertex's children are attached) is
 * an input: the residue X mod 2^64 does not depend on it, but the flag does,
 * because the intermediate tables do.
 *
 * The same DP also runs modulo an odd modulus m < 2^63 (products through
 * 128-bit integers): the map from integers to residues mod m is a ring
 * homomorphism and the DP uses only + and *, so this gives X mod m.  Residues
 * modulo 2^64 and modulo pairwise coprime primes determine X by the Chinese
 * remainder theorem whenever X is below the product of the moduli.
 *
 * Plan format: `child_ptr[t+1]`, `child_idx[t-1]` list, for each template
 * vertex u, its children in attach order (CSR); `root` is the root vertex.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

#define OR_MAXK 16

/* Threads the OpenMP loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- colours */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t index)
{
    uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int oracle_color(uint64_t seed, uint64_t r, uint64_t v, int k)
{
    uint64_t x = oracle_splitmix64(seed, (r << 40) + v);
    return (int)(((u128)x * (u128)(uint64_t)k) >> 64);
}

void oracle_colors(uint64_t seed, uint64_t r, int64_t n, int k, uint8_t *out)
{
    for (int64_t v = 0; v < n; ++v)
        out[v] = (uint8_t)oracle_color(seed, r, (uint64_t)v, k);
}

/* ------------------------------------------------------- Eq. 1 indexing */

static uint64_t binom(int n, int r)
{
    if (r < 0 || n < 0 || r > n) return 0;
    uint64_t b = 1;
    for (int i = 1; i <= r; ++i) b = b * (uint64_t)(n - r + i) / (uint64_t)i;
    return b;
}

/* Eq. 1: the i-th smallest colour c_i (i from 1) contributes binom(c_i, i). */
int64_t oracle_rank(uint32_t mask)
{
    int64_t idx = 0;
    int i = 0;
    for (int c = 0; c < 32; ++c)
        if (mask & (1u << c)) { ++i; idx += (int64_t)binom(c, i); }
    return idx;
}

/* ---------------------------------------------------------- the DP */

typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    int k;
    const uint8_t *col;
    const int32_t *child_ptr;
    const int32_t *child_idx;
    int32_t *rank;          /* rank[mask] by Eq. 1, for every mask of k bits */
    int flag;               /* sticky overflow flag */
    int unpruned;           /* 1: Algorithm-1 order (neighbour loop inside) */
    int oom;
    uint64_t mod;           /* 0: arithmetic mod 2^64 with the flag; else mod this odd m < 2^63 */
} octx;

static uint64_t addm(const octx *c, uint64_t a, uint64_t b)
{
    uint64_t s = a + b;                         /* a, b < m < 2^63: no wrap */
    return s >= c->mod ? s - c->mod : s;
}

static uint64_t mulm(const octx *c, uint64_t a, uint64_t b)
{
    return (uint64_t)(((u128)a * (u128)b) % (u128)c->mod);
}

static int popc(uint32_t x) { return __builtin_popcount(x); }

/* Single-vertex table: W = binom(k,1) = k columns, rank({c}) = c. */
static uint64_t *leaf_table(octx *c)
{
    uint64_t *M = calloc((size_t)c->n * (size_t)c->k, sizeof(uint64_t));
    if (!M) { c->oom = 1; return NULL; }
    for (int64_t v = 0; v < c->n; ++v) M[v * c->k + c->col[v]] = 1;
    return M;
}

/* All (I_s, I_a, I_p) triples of a step with sizes (h, a, p): for every colour
 * set C of size h, every subset C1 of size a, C2 = C \ C1. */
typedef struct { int32_t s, a, p; } triple;

static triple *split_list(octx *c, int h, int a, int64_t *count)
{
    int k = c->k;
    int64_t cnt = (int64_t)binom(k, h) * (int64_t)binom(h, a);
    triple *L = malloc((size_t)(cnt ? cnt : 1) * sizeof(triple));
    if (!L) { c->oom = 1; return NULL; }
    int64_t q = 0;
    for (uint32_t ms = 0; ms < (1u << k); ++ms) {
        if (popc(ms) != h) continue;
        /* every submask of ms */
        for (uint32_t ma = ms;; ma = (ma - 1) & ms) {
            if (popc(ma) == a) {
                L[q].s = c->rank[ms];
                L[q].a = c->rank[ma];
                L[q].p = c->rank[ms ^ ma];
                ++q;
            }
            if (ma == 0) break;
        }
    }
    *count = q;
    return L;
}

/* N = A * M_p : the neighbour sum for every passive column of size p.  Every
 * entry is computed; a carry sets the flag only for the usable entries (colour
 * set without col(v)), see the overflow reading at the top. */
static uint64_t *neighbour_sum(octx *c, const uint64_t *P, int p)
{
    int64_t Wp = (int64_t)binom(c->k, p);
    uint64_t *N = malloc((size_t)c->n * (size_t)Wp * sizeof(uint64_t));
    uint32_t *sets = malloc((size_t)Wp * sizeof(uint32_t));   /* colour set of each column */
    if (!N || !sets) { free(N); free(sets); c->oom = 1; return NULL; }
    for (uint32_t m = 0; m < (1u << c->k); ++m)
        if (popc(m) == p) sets[c->rank[m]] = m;
    int flag = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(|:flag)
    for (int64_t v = 0; v < c->n; ++v) {
        uint64_t *row = N + v * Wp;
        const uint32_t own = 1u << c->col[v];
        for (int64_t q = 0; q < Wp; ++q) row[q] = 0;
        for (int64_t e = c->rp[v]; e < c->rp[v + 1]; ++e) {
            const uint64_t *src = P + (int64_t)c->ci[e] * Wp;
            if (c->mod) {
                for (int64_t q = 0; q < Wp; ++q) row[q] = addm(c, row[q], src[q]);
                continue;
            }
            for (int64_t q = 0; q < Wp; ++q)
                if (__builtin_add_overflow(row[q], src[q], &row[q]) && !(sets[q] & own)) flag = 1;
        }
    }
    c->flag |= flag;
    free(sets);
    return N;
}

/* M_s[v][I_s] = sum over splits of M_a[v][I_a] * N[v][I_p]. */
static uint64_t *combine(octx *c, const uint64_t *Ma, int a, const uint64_t *N, int p)
{
    int h = a + p;
    int64_t Wa = (int64_t)binom(c->k, a), Wp = (int64_t)binom(c->k, p);
    int64_t Ws = (int64_t)binom(c->k, h);
    int64_t cnt;
    triple *L = split_list(c, h, a, &cnt);
    if (!L) return NULL;
    uint64_t *S = calloc((size_t)c->n * (size_t)Ws, sizeof(uint64_t));
    if (!S) { free(L); c->oom = 1; return NULL; }
    int flag = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(|:flag)
    for (int64_t v = 0; v < c->n; ++v) {
        const uint64_t *ra = Ma + v * Wa;
        const uint64_t *rn = N + v * Wp;
        uint64_t *rs = S + v * Ws;
        for (int64_t q = 0; q < cnt; ++q) {
            if (c->mod) {
                rs[L[q].s] = addm(c, rs[L[q].s], mulm(c, ra[L[q].a], rn[L[q].p]));
                continue;
            }
            uint64_t prod;
            flag |= __builtin_mul_overflow(ra[L[q].a], rn[L[q].p], &prod);
            flag |= __builtin_add_overflow(rs[L[q].s], prod, &rs[L[q].s]);
        }
    }
    c->flag |= flag;
    free(L);
    return S;
}

/* Algorithm-1 order: for every split, the neighbour loop runs inside
 * (M_s[v][I_s] += M_a[v][I_a] * M_p[j][I_p] for j in adj(v)).  Used only to
 * cross-check residues; its overflow flag follows different intermediates. */
static uint64_t *combine_unpruned(octx *c, const uint64_t *Ma, int a, const uint64_t *P, int p)
{
    int h = a + p;
    int64_t Wa = (int64_t)binom(c->k, a), Wp = (int64_t)binom(c->k, p);
    int64_t Ws = (int64_t)binom(c->k, h);
    int64_t cnt;
    triple *L = split_list(c, h, a, &cnt);
    if (!L) return NULL;
    uint64_t *S = calloc((size_t)c->n * (size_t)Ws, sizeof(uint64_t));
    if (!S) { free(L); c->oom = 1; return NULL; }
    int flag = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(|:flag)
    for (int64_t v = 0; v < c->n; ++v) {
        const uint64_t *ra = Ma + v * Wa;
        uint64_t *rs = S + v * Ws;
        for (int64_t q = 0; q < cnt; ++q)
            for (int64_t e = c->rp[v]; e < c->rp[v + 1]; ++e) {
                uint64_t prod;
                flag |= __builtin_mul_overflow(ra[L[q].a], P[(int64_t)c->ci[e] * Wp + L[q].p], &prod);
                flag |= __builtin_add_overflow(rs[L[q].s], prod, &rs[L[q].s]);
            }
    }
    c->flag |= flag;
    free(L);
    return S;
}

/* Table of the subtree rooted at u, children attached in plan order. */
static uint64_t *subtree_table(octx *c, int u, int *size_out)
{
    int size = 1;
    uint64_t *M = leaf_table(c);
    if (!M) return NULL;
    for (int32_t e = c->child_ptr[u]; e < c->child_ptr[u + 1]; ++e) {
        int w = c->child_idx[e], p;
        uint64_t *P = subtree_table(c, w, &p);
        if (!P) { free(M); return NULL; }
        uint64_t *S;
        if (c->unpruned) {
            S = combine_unpruned(c, M, size, P, p);
            free(P);
        } else {
            uint64_t *N = neighbour_sum(c, P, p);
            free(P);
            if (!N) { free(M); return NULL; }
            S = combine(c, M, size, N, p);
            free(N);
        }
        free(M);
        if (!S) return NULL;
        M = S;
        size += p;
    }
    *size_out = size;
    return M;
}

static int setup(octx *c, int64_t n, const int64_t *rp, const int32_t *ci, int k,
                 const uint8_t *col, const int32_t *child_ptr, const int32_t *child_idx)
{
    if (k < 1 || k > OR_MAXK) return -1;
    c->n = n; c->rp = rp; c->ci = ci; c->k = k; c->col = col;
    c->child_ptr = child_ptr; c->child_idx = child_idx;
    c->flag = 0; c->unpruned = 0; c->oom = 0; c->mod = 0;
    c->rank = malloc(sizeof(int32_t) << k);
    if (!c->rank) return -2;
    for (uint32_t m = 0; m < (1u << k); ++m) c->rank[m] = (int32_t)oracle_rank(m);
    return 0;
}

/* Root table M_root[v][I(C)], |C| = t: n * binom(k,t) entries into `table`.
 * Returns 0, or <0 on bad input / out of memory.  *flag gets the overflow flag
 * (excluding the final reduction). */
int oracle_root_table(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                      const int32_t *child_ptr, const int32_t *child_idx, int k,
                      const uint8_t *col, int unpruned, uint64_t *table, int *flag)
{
    octx c;
    if (t < 1 || t > k) return -1;
    int rc = setup(&c, n, rp, ci, k, col, child_ptr, child_idx);
    if (rc) return rc;
    c.unpruned = unpruned;
    int size;
    uint64_t *M = subtree_table(&c, root, &size);
    free(c.rank);
    if (!M) return -2;
    if (size != t) { free(M); return -1; }
    memcpy(table, M, (size_t)n * binom(k, t) * sizeof(uint64_t));
    free(M);
    *flag = c.flag;
    return 0;
}

/* X = sum_v sum_{|C|=t} M_root[v][C] for one explicit colouring, modulo 2^64
 * (mod = 0, with the flag) or modulo the odd modulus `mod` < 2^63. */
static int count_colored(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                         const int32_t *child_ptr, const int32_t *child_idx, int k,
                         const uint8_t *col, int unpruned, uint64_t mod, uint64_t *count, int *flag)
{
    octx c;
    if (t < 1 || t > k) return -1;
    if (mod && (mod % 2 == 0 || mod >= (1ULL << 63))) return -1;
    int rc = setup(&c, n, rp, ci, k, col, child_ptr, child_idx);
    if (rc) return rc;
    c.unpruned = unpruned;
    c.mod = mod;
    int size;
    uint64_t *M = subtree_table(&c, root, &size);
    free(c.rank);
    if (!M) return -2;
    if (size != t) { free(M); return -1; }
    int64_t W = (int64_t)binom(k, t);
    uint64_t X = 0;
    int f = c.flag;
    for (int64_t q = 0; q < n * W; ++q) {
        if (mod) X = addm(&c, X, M[q]);
        else f |= __builtin_add_overflow(X, M[q], &X);
    }
    free(M);
    *count = X;
    *flag = mod ? 0 : f;
    return 0;
}

int oracle_count_colored(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                         const int32_t *child_ptr, const int32_t *child_idx, int k,
                         const uint8_t *col, int unpruned, uint64_t *count, int *flag)
{
    return count_colored(n, rp, ci, t, root, child_ptr, child_idx, k, col, unpruned, 0, count, flag);
}

/* X mod `mod` (odd, < 2^63) for one explicit colouring. */
int oracle_count_colored_mod(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                             const int32_t *child_ptr, const int32_t *child_idx, int k,
                             const uint8_t *col, uint64_t mod, uint64_t *count)
{
    int flag;
    return count_colored(n, rp, ci, t, root, child_ptr, child_idx, k, col, 0, mod, count, &flag);
}

/* Colourings first .. first+R-1 from the SplitMix64 colouring rule above;
 * mod = 0: residues mod 2^64 and flags, else residues mod `mod` (flags 0). */
static int count_range(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                       const int32_t *child_ptr, const int32_t *child_idx, int k, uint64_t seed,
                       uint64_t first, int32_t R, uint64_t mod, uint64_t *counts, uint8_t *flags)
{
    uint8_t *col = malloc((size_t)(n ? n : 1));
    if (!col) return -2;
    for (int32_t r = 0; r < R; ++r) {
        oracle_colors(seed, first + (uint64_t)r, n, k, col);
        int f;
        int rc = count_colored(n, rp, ci, t, root, child_ptr, child_idx, k, col, 0, mod, &counts[r], &f);
        if (rc) { free(col); return rc; }
        if (flags) flags[r] = (uint8_t)f;
    }
    free(col);
    return 0;
}

int oracle_count(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                 const int32_t *child_ptr, const int32_t *child_idx, int k, uint64_t seed,
                 uint64_t first, int32_t R, uint64_t *counts, uint8_t *flags)
{
    return count_range(n, rp, ci, t, root, child_ptr, child_idx, k, seed, first, R, 0, counts, flags);
}

int oracle_count_mod(int64_t n, const int64_t *rp, const int32_t *ci, int t, int root,
                     const int32_t *child_ptr, const int32_t *child_idx, int k, uint64_t seed,
                     uint64_t first, int32_t R, uint64_t mod, uint64_t *counts)
{
    return count_range(n, rp, ci, t, root, child_ptr, child_idx, k, seed, first, R, mod, counts, NULL);
}
