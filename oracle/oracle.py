"""Python face of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrappers around ``liboracle.so`` (built from ``oracle.c`` by
``oracle/build.py``) plus the parts of the method that are plain host
arithmetic on the template alone:

* ``aut(t, edges)``: the automorphism count of the template tree (needed to
  turn colourful *maps* into subgraph *copies*; the paper counts embeddings,
  Section 2.1);
* ``colorful_probability(k, t)``: the probability that a fixed injective map is
  colourful, k!/((k-t)! k^t), which is k!/k^k for k = t (Section 2.1, phase 1);
* ``estimate(counts, k, t, aut)``: the colour-coding estimates.

The plan passed to the counting calls is a rooted, ordered tree:
``root`` and ``children[u]`` = the children of u in the order they are attached
(each attach is one DP step with active child = what u has so far and passive
child = the subtree of the attached vertex; Section 2.1, phase 2).
"""
from __future__ import annotations

import ctypes
import math
import os
from collections import Counter

import numpy as np

__all__ = [
    "lib", "splitmix64", "color", "colors", "rank", "plan_arrays", "root_plan",
    "count", "count_colored", "root_table", "aut", "colorful_probability",
    "estimate", "binom", "threads", "count_colored_mod", "count_mod", "PRIMES", "crt",
    "count_exact",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib():
    """Load liboracle.so (built by oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is missing: run `python oracle/build.py`")
        L = ctypes.CDLL(_LIB)
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_threads.argtypes = []
        L.oracle_splitmix64.restype = ctypes.c_uint64
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_color.restype = ctypes.c_int
        L.oracle_color.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.oracle_colors.restype = None
        L.oracle_colors.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, _u8p]
        L.oracle_rank.restype = ctypes.c_int64
        L.oracle_rank.argtypes = [ctypes.c_uint32]
        common = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int]
        L.oracle_root_table.restype = ctypes.c_int
        L.oracle_root_table.argtypes = common + [_u8p, ctypes.c_int, _u64p, ctypes.POINTER(ctypes.c_int)]
        L.oracle_count_colored.restype = ctypes.c_int
        L.oracle_count_colored.argtypes = common + [_u8p, ctypes.c_int, _u64p, ctypes.POINTER(ctypes.c_int)]
        L.oracle_count.restype = ctypes.c_int
        L.oracle_count.argtypes = common + [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, _u64p, _u8p]
        L.oracle_count_colored_mod.restype = ctypes.c_int
        L.oracle_count_colored_mod.argtypes = common + [_u8p, ctypes.c_uint64, _u64p]
        L.oracle_count_mod.restype = ctypes.c_int
        L.oracle_count_mod.argtypes = common + [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                                ctypes.c_uint64, _u64p]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def binom(n: int, r: int) -> int:
    return math.comb(n, r) if 0 <= r <= n else 0


def splitmix64(seed: int, index: int) -> int:
    return int(lib().oracle_splitmix64(seed & (2**64 - 1), index & (2**64 - 1)))


def color(seed: int, r: int, v: int, k: int) -> int:
    return int(lib().oracle_color(seed, r, v, k))


def colors(seed: int, r: int, n: int, k: int) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=np.uint8)
    lib().oracle_colors(seed, r, n, k, _ptr(out, _u8p))
    return out[:n]


def rank(mask: int) -> int:
    """Eq. 1 index of the colour set given as a bitmask."""
    return int(lib().oracle_rank(mask))


def root_plan(t: int, edges, root: int, order: str = "given"):
    """Rooted ordered tree from an edge list: children[u] in the order given by
    `order` ("given": edge-list order; "small": by ascending subtree size;
    "large": descending)."""
    adj = [[] for _ in range(t)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    children = [[] for _ in range(t)]
    parent = [-1] * t
    seen = [False] * t
    stack = [root]
    seen[root] = True
    orderv = []
    while stack:
        u = stack.pop()
        orderv.append(u)
        for w in adj[u]:
            if not seen[w]:
                seen[w] = True
                parent[w] = u
                children[u].append(w)
                stack.append(w)
    if not all(seen):
        raise ValueError("template is not connected")
    size = [1] * t
    for u in reversed(orderv):
        if parent[u] >= 0:
            size[parent[u]] += size[u]
    if order == "small":
        for u in range(t):
            children[u].sort(key=lambda w: (size[w], w))
    elif order == "large":
        for u in range(t):
            children[u].sort(key=lambda w: (-size[w], w))
    return root, children


def plan_arrays(t: int, root: int, children):
    """CSR form (child_ptr[t+1], child_idx[t-1]) of a rooted ordered tree."""
    ptr = np.zeros(t + 1, dtype=np.int32)
    idx = []
    for u in range(t):
        idx.extend(children[u])
        ptr[u + 1] = len(idx)
    return int(root), ptr, np.asarray(idx if idx else [0], dtype=np.int32)


def _csr_args(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(g.col_idx if g.col_idx.size else np.zeros(1, np.int32), dtype=np.int32)
    return rp, ci


def count_colored(g, t: int, plan, k: int, col, unpruned: bool = False):
    """(X mod 2^64, overflow flag) for one explicit colouring `col` (uint8[n])."""
    root, children = plan
    root, ptr, idx = plan_arrays(t, root, children)
    rp, ci = _csr_args(g)
    col = np.ascontiguousarray(col, dtype=np.uint8)
    if col.size == 0:
        col = np.zeros(1, np.uint8)
    X = ctypes.c_uint64(0)
    f = ctypes.c_int(0)
    rc = lib().oracle_count_colored(g.n, _ptr(rp, _i64p), _ptr(ci, _i32p), t, root,
                                    _ptr(ptr, _i32p), _ptr(idx, _i32p), k, _ptr(col, _u8p),
                                    int(unpruned), ctypes.byref(X), ctypes.byref(f))
    if rc:
        raise RuntimeError(f"oracle_count_colored failed ({rc})")
    return int(X.value), int(f.value)


def root_table(g, t: int, plan, k: int, col, unpruned: bool = False):
    """(M_root as uint64[n, binom(k,t)], flag) for one explicit colouring."""
    root, children = plan
    root, ptr, idx = plan_arrays(t, root, children)
    rp, ci = _csr_args(g)
    col = np.ascontiguousarray(col, dtype=np.uint8)
    W = binom(k, t)
    out = np.zeros((max(g.n, 1), W), dtype=np.uint64)
    f = ctypes.c_int(0)
    rc = lib().oracle_root_table(g.n, _ptr(rp, _i64p), _ptr(ci, _i32p), t, root,
                                 _ptr(ptr, _i32p), _ptr(idx, _i32p), k, _ptr(col, _u8p),
                                 int(unpruned), _ptr(out, _u64p), ctypes.byref(f))
    if rc:
        raise RuntimeError(f"oracle_root_table failed ({rc})")
    return out[:g.n], int(f.value)


def count(g, t: int, plan, k: int, seed: int, first: int, R: int):
    """Per-colouring (counts uint64[R], flags uint8[R]) for colourings
    first..first+R-1 drawn by the SplitMix64 colouring rule."""
    root, children = plan
    root, ptr, idx = plan_arrays(t, root, children)
    rp, ci = _csr_args(g)
    counts = np.zeros(max(R, 1), dtype=np.uint64)
    flags = np.zeros(max(R, 1), dtype=np.uint8)
    rc = lib().oracle_count(g.n, _ptr(rp, _i64p), _ptr(ci, _i32p), t, root,
                            _ptr(ptr, _i32p), _ptr(idx, _i32p), k,
                            seed & (2**64 - 1), first, R, _ptr(counts, _u64p), _ptr(flags, _u8p))
    if rc:
        raise RuntimeError(f"oracle_count failed ({rc})")
    return counts[:R], flags[:R]


def count_colored_mod(g, t: int, plan, k: int, col, mod: int) -> int:
    """X mod `mod` (odd, < 2^63) for one explicit colouring."""
    root, children = plan
    root, ptr, idx = plan_arrays(t, root, children)
    rp, ci = _csr_args(g)
    col = np.ascontiguousarray(col, dtype=np.uint8)
    if col.size == 0:
        col = np.zeros(1, np.uint8)
    X = ctypes.c_uint64(0)
    rc = lib().oracle_count_colored_mod(g.n, _ptr(rp, _i64p), _ptr(ci, _i32p), t, root,
                                        _ptr(ptr, _i32p), _ptr(idx, _i32p), k, _ptr(col, _u8p),
                                        mod, ctypes.byref(X))
    if rc:
        raise RuntimeError(f"oracle_count_colored_mod failed ({rc})")
    return int(X.value)


def count_mod(g, t: int, plan, k: int, seed: int, first: int, R: int, mod: int):
    """Per-colouring residues mod `mod` (odd, < 2^63) for colourings first..first+R-1."""
    root, children = plan
    root, ptr, idx = plan_arrays(t, root, children)
    rp, ci = _csr_args(g)
    counts = np.zeros(max(R, 1), dtype=np.uint64)
    rc = lib().oracle_count_mod(g.n, _ptr(rp, _i64p), _ptr(ci, _i32p), t, root,
                                _ptr(ptr, _i32p), _ptr(idx, _i32p), k,
                                seed & (2**64 - 1), first, R, mod, _ptr(counts, _u64p))
    if rc:
        raise RuntimeError(f"oracle_count_mod failed ({rc})")
    return counts[:R]


# Odd primes below 2^63 that serve as extra moduli beside 2^64.
PRIMES = (2**61 - 1, 2**62 - 57, 2**63 - 25)


def crt(residues, moduli):
    """The unique x in [0, prod(moduli)) with x = residues[i] mod moduli[i]
    (pairwise coprime moduli), by incremental Chinese remaindering."""
    x, m = 0, 1
    for a, mi in zip(residues, moduli):
        t = ((int(a) - x) * pow(m, -1, mi)) % mi
        x += m * t
        m *= mi
    return x


def count_exact(g, t: int, plan, k: int, seed: int, first: int, R: int, n_primes: int = 3):
    """Per-colouring X mod 2^64 * PRIMES[0] * ... * PRIMES[n_primes-1] (Python
    ints), from the residue DPs; X itself whenever it is below that product."""
    moduli = [2**64] + list(PRIMES[:n_primes])
    res = [count(g, t, plan, k, seed, first, R)[0]]
    res += [count_mod(g, t, plan, k, seed, first, R, p) for p in PRIMES[:n_primes]]
    return [crt([int(r[i]) for r in res], moduli) for i in range(R)]


# ------------------------------------------------------------ template-only math

def _centers(t, adj):
    deg = [len(a) for a in adj]
    layer = [u for u in range(t) if deg[u] <= 1]
    remaining = t
    removed = [False] * t
    while remaining > 2:
        remaining -= len(layer)
        nxt = []
        for u in layer:
            removed[u] = True
            for w in adj[u]:
                if not removed[w]:
                    deg[w] -= 1
                    if deg[w] == 1:
                        nxt.append(w)
        layer = nxt
    return [u for u in range(t) if not removed[u]]


def _rooted_form(u, parent, adj):
    """(canonical form, automorphisms fixing u) of the subtree at u (AHU)."""
    forms = []
    autc = 1
    for w in adj[u]:
        if w != parent:
            f, a = _rooted_form(w, u, adj)
            forms.append(f)
            autc *= a
    for mult in Counter(forms).values():
        autc *= math.factorial(mult)
    return "(" + "".join(sorted(forms)) + ")", autc


def aut(t: int, edges) -> int:
    """Number of automorphisms of the (unrooted) template tree."""
    if t <= 1:
        return 1
    adj = [[] for _ in range(t)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    cs = _centers(t, adj)
    if len(cs) == 1:
        return _rooted_form(cs[0], -1, adj)[1]
    c1, c2 = cs
    f1, a1 = _rooted_form(c1, c2, adj)
    f2, a2 = _rooted_form(c2, c1, adj)
    return a1 * a2 * (2 if f1 == f2 else 1)


def colorful_probability(k: int, t: int) -> float:
    """P(a fixed injective map of t vertices is colourful) = k!/((k-t)! k^t)."""
    return math.factorial(k) / (math.factorial(k - t) * k ** t)


def estimate(counts, flags, k: int, t: int, aut_t: int):
    """(estimated maps, estimated copies); NaN if any colouring overflowed."""
    if len(counts) == 0 or any(int(f) for f in flags):
        return float("nan"), float("nan")
    mean = float(np.mean(np.asarray(counts, dtype=np.float64)))
    maps = mean / colorful_probability(k, t)
    return maps, maps / aut_t
