"""Writes tests/golden/full_size.json: oracle residues and overflow flags for
sampled colourings of the full-size workloads, and, with --exact, the exact
counts of the sampled colourings that overflowed (Chinese remaindering of the
oracle's residues mod 2^64 and mod three primes).

Calls only the CPU oracle (oracle/) and the seeded input generators; nothing
here touches the HIP library.  Each entry names its generator call, template,
explicit plan (root and ordered children, so the flag is comparable), k,
seed and the colourings computed.  Run on a host with enough memory (the
k = 12 entries hold up to ~80 GB of tables at once):

    python tests/golden/make_full_size.py [--out PATH] [--exact] [names...]

Entries already present are kept; results are written after each colouring.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from paper_1903_04395_amd import inputs as I         # noqa: E402

OUT = os.path.join(HERE, "full_size.json")

# name: (graph generator call, template, root, k, seed, colourings to compute)
ENTRIES = {
    "er2000_p5_k5": (("erdos_renyi", (2000, 10000), {"seed": 1}), ("path", 5), 0, 5, 2024, list(range(64))),
    "rmat20_tree10_k10": (("rmat", (20, 16), {"seed": 0}), ("prufer", 10, 0), 0, 10, 1, list(range(8))),
    "chunglu4m_tree12_k12": (("chung_lu", (4194304, 30, 2.1), {"seed": 3}), ("prufer", 12, 3), 0, 12, 7,
                             list(range(16))),
    # every colouring of the star is also checked against its closed form
    "chunglu4m_star12_k12": (("chung_lu", (4194304, 30, 2.1), {"seed": 3}), ("star", 12), 0, 12, 7, [0, 15]),
    "rmat19_tree15_k15": (("rmat", (19, 16), {"seed": 4}), ("prufer", 15, 4), 0, 15, 9, list(range(4))),
}


def make_graph(spec):
    fn, args, kw = spec
    return getattr(I, fn)(*args, **kw)


def make_tree(spec):
    if spec[0] == "path":
        return spec[1], I.path(spec[1])
    if spec[0] == "star":
        return spec[1], I.star(spec[1])
    return spec[1], I.prufer_tree(spec[1], spec[2])


def main(names, out=OUT, exact=False):
    data = json.load(open(out)) if os.path.exists(out) else {}
    graphs = {}
    for name in names:
        gspec, tspec, root, k, seed, cols = ENTRIES[name]
        key = json.dumps(gspec)
        if key not in graphs:
            t0 = time.time()
            graphs = {key: make_graph(gspec)}
            print(f"[golden] graph {gspec}: {graphs[key]} in {time.time() - t0:.0f}s", flush=True)
        g = graphs[key]
        t, edges = make_tree(tspec)
        rt, children = O.root_plan(t, edges, root, "small")
        entry = data.get(name) or {
            "graph": {"fn": gspec[0], "args": list(gspec[1]), "kwargs": gspec[2]},
            "template_edges": [list(e) for e in edges], "t": t, "root": rt, "children": children,
            "k": k, "seed": seed, "results": {}}
        for r in cols:
            if str(r) in entry["results"]:
                continue
            t0 = time.time()
            c, f = O.count(g, t, (rt, children), k, seed, r, 1)
            entry["results"][str(r)] = [str(int(c[0])), int(f[0])]
            data[name] = entry
            with open(out + ".tmp", "w") as fh:
                json.dump(data, fh, indent=1)
            os.replace(out + ".tmp", out)
            print(f"[golden] {name} colouring {r}: {int(c[0])} flag {int(f[0])} "
                  f"({time.time() - t0:.0f}s, {O.threads()} threads)", flush=True)
        if not exact:
            continue
        ex = entry.setdefault("exact", {})
        for r in cols:
            if str(r) in ex or not entry["results"][str(r)][1]:
                continue
            t0 = time.time()
            res = [int(entry["results"][str(r)][0])]
            res += [int(O.count_mod(g, t, (rt, children), k, seed, r, 1, p)[0]) for p in O.PRIMES]
            ex[str(r)] = str(O.crt(res, [2**64] + list(O.PRIMES)))
            data[name] = entry
            with open(out + ".tmp", "w") as fh:
                json.dump(data, fh, indent=1)
            os.replace(out + ".tmp", out)
            print(f"[golden] {name} colouring {r}: exact {ex[str(r)]} ({time.time() - t0:.0f}s)", flush=True)


if __name__ == "__main__":
    argv = sys.argv[1:]
    out = OUT
    if argv[:1] == ["--out"]:
        out, argv = argv[1], argv[2:]
    exact = "--exact" in argv
    argv = [a for a in argv if a != "--exact"]
    main(argv or list(ENTRIES), out, exact)
