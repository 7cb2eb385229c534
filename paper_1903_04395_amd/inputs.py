"""Seeded synthetic inputs: graphs (CSR) and template trees.

This module produces *inputs only*. It holds none of the counting method's
arithmetic (no colour sets, no tables, no counts), so both the HIP path and the
CPU oracle can be fed from it without sharing any of the method's code.

Graphs are simple and undirected and are returned as a symmetric 0/1 adjacency
in CSR form (``row_ptr`` int64 of length n+1, ``col_idx`` int32 of length nnz,
rows sorted, no duplicates, no self-loops), which is the adjacency-matrix form
the paper builds its SpMM on (Section 4.3).

Generators (all seeded through ``numpy.random.Generator(PCG64(seed))``):

* ``erdos_renyi(n, m, seed)`` -- G(n, m): m distinct unordered pairs, uniform.
* ``rmat(scale, edge_factor, a, b, c, seed)`` -- the R-MAT recursive model
  (Chakrabarti, Zhan, Faloutsos 2004) with Graph500's defaults; the paper's
  GS20-22 and RMAT datasets come from it (Table 3).  Edges are symmetrised,
  deduplicated and self-loops removed; vertex labels are randomly permuted as in
  the Graph500 generator.
* ``chung_lu(n, avg_deg, gamma, seed)`` -- expected-degree power-law graph with
  weights w_i proportional to (i+1)^(-1/(gamma-1)), capped at sqrt(n*avg_deg);
  stands in for the paper's power-law social graphs (Table 3).
* ``prufer_tree(t, seed)``, ``star(t)``, ``path(t)`` -- template trees as edge
  lists over vertices 0..t-1.
* ``serving_queries(nq, qps, seed)`` -- a Poisson stream of counting queries
  over three resident graphs.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR", "csr_from_edges", "erdos_renyi", "rmat", "chung_lu",
    "prufer_tree", "prufer_decode", "star", "path", "random_small_graph",
    "degree_stats", "serving_queries",
]


class CSR:
    """Symmetric adjacency in CSR form (n vertices, nnz directed entries)."""

    __slots__ = ("n", "row_ptr", "col_idx")

    def __init__(self, n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self):
        """Undirected edge list (u < v) as an (m, 2) int64 array."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def __repr__(self):
        return f"CSR(n={self.n}, nnz={self.nnz})"


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Symmetrise, drop self-loops and duplicates, and build a sorted CSR."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique(a * n + b)          # sorted by (row, col), deduplicated
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, cols)


def erdos_renyi(n: int, m: int, seed: int) -> CSR:
    """G(n, m): exactly m distinct unordered pairs {u, v}, u != v, uniform."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges for a simple graph")
    rng = np.random.Generator(np.random.PCG64(seed))
    have = np.empty(0, dtype=np.int64)
    while have.size < m:
        need = m - have.size
        u = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        v = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = u != v
        lo = np.minimum(u[ok], v[ok])
        hi = np.maximum(u[ok], v[ok])
        cand = lo * n + hi
        # keep first occurrences in draw order so the result is a function of the seed
        allk = np.concatenate([have, cand])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        have = allk[first][:m]
    lo = have // n
    hi = have - lo * n
    return csr_from_edges(n, lo, hi)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, permute: bool = True) -> CSR:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale sampled edges."""
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    chunk = 1 << 22
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        rs = np.zeros(e - s, dtype=np.int64)
        cs = np.zeros(e - s, dtype=np.int64)
        for _ in range(scale):
            u = rng.random(e - s)
            rbit = u >= ab                       # quadrants c, d -> lower half
            cbit = ((u >= a) & (u < ab)) | (u >= abc)   # quadrants b, d -> right half
            rs = (rs << 1) | rbit
            cs = (cs << 1) | cbit
        src[s:e] = rs
        dst[s:e] = cs
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    return csr_from_edges(n, src, dst)


def chung_lu(n: int, avg_deg: float, gamma: float, seed: int,
             cap: float | None = None, permute: bool = True) -> CSR:
    """Chung-Lu graph: n*avg_deg/2 endpoint pairs drawn with P(i) ~ w_i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= avg_deg * n / w.sum()
    if cap is None:
        cap = float(np.sqrt(n * avg_deg))
    w = np.minimum(w, cap)
    p = w / w.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    m = int(round(n * avg_deg / 2))
    src = np.searchsorted(cdf, rng.random(m), side="right").astype(np.int64)
    dst = np.searchsorted(cdf, rng.random(m), side="right").astype(np.int64)
    np.minimum(src, n - 1, out=src)
    np.minimum(dst, n - 1, out=dst)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    return csr_from_edges(n, src, dst)


def random_small_graph(n: int, p: float, seed: int) -> CSR:
    """G(n, p) for tiny brute-force tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return csr_from_edges(n, iu[keep], ju[keep])


def prufer_decode(seq, t: int):
    """Decode a Pruefer sequence of length t-2 into the t-1 edges of a labelled tree."""
    seq = [int(x) for x in seq]
    if t == 1:
        return []
    if t == 2:
        return [(0, 1)]
    degree = [1] * t
    for x in seq:
        degree[x] += 1
    edges = []
    for x in seq:
        leaf = min(i for i in range(t) if degree[i] == 1)
        edges.append((leaf, x))
        degree[leaf] -= 1
        degree[x] -= 1
    rest = [i for i in range(t) if degree[i] == 1]
    edges.append((rest[0], rest[1]))
    return edges


def prufer_tree(t: int, seed: int):
    """Uniformly random labelled tree on t vertices from a seeded Pruefer sequence."""
    rng = np.random.Generator(np.random.PCG64(seed))
    seq = rng.integers(0, t, size=max(t - 2, 0))
    return prufer_decode(seq, t)


def star(t: int):
    """Star K_{1,t-1}: centre 0, leaves 1..t-1."""
    return [(0, i) for i in range(1, t)]


def path(t: int):
    """Path on t vertices 0-1-...-(t-1)."""
    return [(i, i + 1) for i in range(t - 1)]


def degree_stats(g: CSR) -> dict:
    d = g.degrees()
    nz = d[d > 0]
    return {
        "n": g.n, "nnz": g.nnz, "non_isolated": int(nz.size),
        "avg_deg": float(nz.mean()) if nz.size else 0.0,
        "max_deg": int(d.max()) if d.size else 0,
        "p99_deg": float(np.percentile(d, 99)) if d.size else 0.0,
    }


def serving_queries(nq: int, qps: float = 200.0, seed: int = 2019):
    """A seeded Poisson query stream over three resident graphs: arrival time
    (seconds, exponential gaps at `qps`), graph index 0..2, a Pruefer tree of
    3..12 vertices (its own seed), k = t, 1..32 colourings, colouring seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, at = [], 0.0
    for i in range(nq):
        at += rng.exponential(1.0 / qps)
        t = int(rng.integers(3, 13))
        out.append({"at": at, "graph": int(rng.integers(0, 3)), "t": t, "edges": prufer_tree(t, 10_000 + i),
                    "n": int(rng.integers(1, 33)), "seed": int(rng.integers(0, 1 << 40))})
    return out
