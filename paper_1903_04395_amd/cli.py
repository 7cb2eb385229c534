"""Command line: count a tree template in a graph from edge-list files.

    python -m paper_1903_04395_amd.cli --graph G.txt --template T.txt [--k K]
        (--colorings R | --eps E --delta D [--max-colorings M])
        [--seed S] [--first F] [--device 0]

Both files are whitespace-separated vertex pairs, one edge per line; blank
lines and lines starting with '#' or '%' are skipped.  Graph vertex ids are
non-negative integers (the graph has max id + 1 vertices; it is symmetrised and
loops and duplicate edges are dropped, since the method counts in simple
undirected graphs).  The template must be a tree on vertices 0..t-1.  k
defaults to t.

With --colorings R the library runs colourings F..F+R-1 with exact counts
(sc_run_exact) and reports their mean estimate; with --eps/--delta it runs the
median-of-means rule (sc_estimate, sample-variance mode unless --bound).  The
result is one JSON object on stdout.  Every count is computed by libsc's HIP
kernels; this module only reads files and marshals arguments.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs


def read_pairs(path: str) -> np.ndarray:
    """Integer vertex pairs of an edge-list file, shape (m, 2)."""
    rows = []
    with open(path) as fh:
        for ln, line in enumerate(fh, 1):
            s = line.strip()
            if not s or s[0] in "#%":
                continue
            parts = s.split()
            if len(parts) < 2:
                raise ValueError(f"{path}:{ln}: expected two vertex ids")
            u, v = int(parts[0]), int(parts[1])
            if u < 0 or v < 0:
                raise ValueError(f"{path}:{ln}: negative vertex id")
            rows.append((u, v))
    return np.asarray(rows, dtype=np.int64).reshape(-1, 2)


def graph_from_pairs(pairs: np.ndarray, n: int | None = None) -> inputs.CSR:
    """Simple undirected CSR over max id + 1 vertices (or n)."""
    if n is None:
        n = int(pairs.max()) + 1 if pairs.size else 1
    if pairs.size and int(pairs.max()) >= n:
        raise ValueError("vertex id out of range")
    return inputs.csr_from_edges(n, pairs[:, 0], pairs[:, 1])


def template_from_pairs(pairs: np.ndarray) -> tuple[int, np.ndarray]:
    """(t, edges) of a tree on vertices 0..t-1; raises if it is not one."""
    t = int(pairs.max()) + 1 if pairs.size else 1
    if len(pairs) != t - 1:
        raise ValueError(f"a tree on {t} vertices has {t - 1} edges, got {len(pairs)}")
    parent = list(range(t))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for u, v in pairs:
        ru, rv = find(int(u)), find(int(v))
        if ru == rv:
            raise ValueError("template has a cycle or a repeated edge")
        parent[ru] = rv
    return t, pairs.astype(np.int32)


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--graph", required=True)
    ap.add_argument("--template", required=True)
    ap.add_argument("--k", type=int, default=0, help="colours (default: template size)")
    ap.add_argument("--colorings", type=int, default=0)
    ap.add_argument("--eps", type=float, default=0.0)
    ap.add_argument("--delta", type=float, default=0.05)
    ap.add_argument("--bound", action="store_true", help="with --eps: the variance bound, not the sample")
    ap.add_argument("--max-colorings", type=int, default=0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--device", type=int, default=0)
    a = ap.parse_args(argv)
    if (a.colorings > 0) == (a.eps > 0):
        ap.error("give exactly one of --colorings or --eps")
    return a


def main(argv=None) -> dict:
    a = parse(argv)
    from . import sc                                   # loads libsc (needs the built library)
    g = graph_from_pairs(read_pairs(a.graph))
    t, edges = template_from_pairs(read_pairs(a.template))
    k = a.k or t
    out = {"graph": {"n": g.n, "nnz": g.nnz}, "t": t, "k": k, "seed": a.seed}
    with sc.Context(a.device) as ctx:
        gid = ctx.load_graph(g)
        tid = ctx.load_template(t, edges)
        ctx.set_colors(k, a.seed)
        if a.colorings > 0:
            counts, exact, hom, maps, copies = ctx.run_exact(gid, tid, a.first, a.colorings)
            out.update({"colorings": a.colorings, "first": a.first, "exact": bool(exact.all()),
                        "mean_count": float(np.mean([float(c) for c in counts])) if counts else 0.0,
                        "est_maps": maps, "est_copies": copies, "hom_bound": hom})
        else:
            mode = sc.SC_EST_BOUND if a.bound else sc.SC_EST_SAMPLE
            e = ctx.estimate(gid, tid, a.eps, a.delta, mode, a.max_colorings, a.first)
            out.update({"eps": a.eps, "delta": a.delta, "mode": "bound" if a.bound else "sample",
                        "colorings": e.colorings, "groups": e.groups, "per_group": e.per_group,
                        "needed": e.needed, "exact": bool(e.exact), "est_maps": e.est_maps,
                        "est_copies": e.est_copies, "mean_maps": e.mean_maps, "rel_stderr": e.rel_stderr})
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main(sys.argv[1:])
