"""Benchmark: colour-coding tree counting on one MI355X.

Workload (the largest single-GPU configuration): a Chung-Lu power-law graph
(4,194,304 vertices, mean degree 30, degree exponent 2.1, weights capped at
sqrt(n * mean degree), seed 3; symmetrised, deduplicated, self-loops removed,
labels permuted), counted against two 12-vertex templates -- a tree from a
seeded Pruefer sequence (seed 3) and the 12-star -- with k = 12 colours and 16
colourings of each template per step.  One "step" is one sc_run of 16
colourings of the tree and one of 16 colourings of the star (colouring, every
DP step, root reduction, 9-byte-per-colouring result copy; the library splits
each into the passes that fit HBM); the graph is resident in HBM before the
timed region starts.

Prints one JSON line.  `value` is G-updates/s: per colouring the neighbour-sum
updates sum_steps nnz*C(k,p) plus the multiply-adds sum_steps n*C(k,h)*C(h,a)
(n*C(k,h) for a select step), summed over both templates and the timed
colourings, over the timed wall time.  `roofline` describes the DP step (the
split pre-pass and row kernel of each step, 99.9% of the GPU time) from HIP
events recorded by libsc on its stream around every launch in the timed
region, with the compulsory bytes of the paper's table layout; `steps` gives
each DP step's time against both roofs it could meet (HBM bytes, and the
multiply-adds at the vector-ALU rate measured by sc_valu_probe).
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload:
the first three DP steps of both templates' plans (the 4-vertex star rooted at
its centre, k = 12) for one colouring on the whole graph, and checks that
sample's residue and flag against the GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip sc_autotune of both templates before the timed region")
    ap.add_argument("--tune-save", default=None, help="write the autotuner's picks to this file (sc_tune_save)")
    ap.add_argument("--tune-load", default=None,
                    help="load tuning from this file (sc_tune_load) instead of running the autotuner")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (RMAT-20 workload, plain vs batched, exact counts)")
    ap.add_argument("--opt", action="append", default=[], help="libsc option NUM=VALUE (ablation)")
    ap.add_argument("--breakdown", action="store_true", help="also print the per-family table")
    ap.add_argument("--configs", action="store_true",
                    help="timings of the other configurations (ER 2000 / Chung-Lu 4M k=12 / RMAT-19 k=15)")
    ap.add_argument("--only", default=None, help="with --configs: run only the named configuration")
    ap.add_argument("--no-tune", action="store_true", help="with --configs: skip the autotuner")
    ap.add_argument("--gather-probe", action="store_true",
                    help="only time whole-row gathers in RMAT-20 and Chung-Lu neighbour order, and streaming "
                         "copy and read rates")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--forms", action="store_true",
                    help="plain per-colouring launch loop vs batched form (config 1 and the headline workload)")
    ap.add_argument("--exact", action="store_true",
                    help="time exact wide counts (uint64 pass + residue passes + CRT) beside the uint64 "
                         "pass, on the RMAT scale-20 and Chung-Lu k=12 workloads")
    ap.add_argument("--ablation", action="store_true",
                    help="pruning ablation: FASCIA and PFASCIA baseline kernels beside the library's path, "
                         "RMAT scale 16, Pruefer trees of 6..10 vertices, k = t, one colouring")
    ap.add_argument("--serve", action="store_true",
                    help="serving mix: RMAT 18/20/22 resident, Poisson query stream, p50/p99 latency")
    ap.add_argument("--queries", type=int, default=40, help="stream length for --serve")
    ap.add_argument("--qps", type=float, default=200.0, help="offered queries/s for --serve")
    ap.add_argument("--streams", type=int, default=4, help="streams of the serving loop for --serve")
    return ap.parse_args()


def timed(fn):
    """Wall time of fn(); sc_run returns only after its results are on the host."""
    t0 = time.perf_counter()
    out = fn()
    return time.perf_counter() - t0, out


def forms_bench():
    """Colourings/s of the plain per-colouring launch loop (one colouring per
    sc_run call, no folding) against the batched form (colourings folded into
    the columns, each pass replayed from a captured hipGraph, one host wait per
    call; then the whole call replayed from one graph), on the same colourings;
    results must agree."""
    import numpy as np
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    out = {}
    ctx = sc.Context(0)
    g20 = I.rmat(20, 16, seed=0)
    cases = [("er2000-p5-k5", I.erdos_renyi(2000, 10000, seed=1), 5, I.path(5), 0, 256, 64),
             ("rmat20-tree10-k10", g20, 10, I.prufer_tree(10, 0), -1, 16, 8),
             ("rmat20-tree10-k10-b16", g20, 10, I.prufer_tree(10, 0), -1, 32, 16)]
    for name, g, t, edges, root, R, B in cases:
        gid = ctx.load_graph(g)
        tid = ctx.load_template(t, edges, root)
        ctx.set_colors(t, 1)
        # plain: one colouring per call
        ctx.set_option(sc.SC_OPT_MAX_BATCH, 1)
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
        ctx.run(gid, tid, 0, 1)
        dt_p, plain = timed(lambda: [ctx.run(gid, tid, r, 1)[0][0] for r in range(R)])
        # batched: B colourings per pass, hipGraph replay per pass, then one
        # graph for the whole call
        ctx.set_option(sc.SC_OPT_MAX_BATCH, B)
        ctx.set_option(sc.SC_OPT_GRAPH, 1)
        ctx.run(gid, tid, 0, R)
        dt_b, (cb, _, _, _) = timed(lambda: ctx.run(gid, tid, 0, R))
        ctx.set_option(sc.SC_OPT_GRAPH, 2)
        ctx.run(gid, tid, 0, R)
        dt_g, (cg, _, _, _) = timed(lambda: ctx.run(gid, tid, 0, R))
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
        ctx.set_option(sc.SC_OPT_MAX_BATCH, 64)
        assert np.array_equal(np.asarray(plain, np.uint64), cb), name
        assert np.array_equal(cg, cb), name
        out[name] = {"colorings": R, "batch": B, "plain_colorings_per_s": round(R / dt_p, 1),
                     "batched_colorings_per_s": round(R / dt_b, 1), "ratio": round(dt_p / dt_b, 2),
                     "one_graph_colorings_per_s": round(R / dt_g, 1)}
        print(f"[bench] forms {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.unload_graph(gid)
    ctx.close()
    print(json.dumps({"forms": out}), flush=True)


def serve_bench(nq, qps=200.0, streams=4):
    """The serving mix: three resident RMAT graphs (scale 18, 20, 22; 16
    edges/vertex), a seeded Poisson stream (200 queries/s by default) of
    (random graph, random 3-12-vertex Pruefer tree, k = t, 1-32 colourings),
    admission by a 200 GB table budget, four streams by default.  Latency =
    submit to result."""
    import numpy as np
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    ctx = sc.Context(0)
    gids = []
    for scale in (18, 20, 22):
        tg = time.time()
        g = I.rmat(scale, 16, seed=scale)
        gids.append(ctx.load_graph(g))
        print(f"[bench] serve graph scale {scale}: n={g.n} nnz={g.nnz} ({time.time() - tg:.0f}s)",
              file=sys.stderr, flush=True)
        del g
    qs = I.serving_queries(nq, qps, seed=2019)
    tids = [ctx.load_template(q["t"], q["edges"]) for q in qs]
    ctx.serve_start(mem_budget_bytes=200 * 10**9, max_inflight=streams, max_batch=64)
    pending = {}
    results = []
    t0 = time.perf_counter()
    i = 0
    while i < nq or pending:
        now = time.perf_counter() - t0
        while i < nq and qs[i]["at"] <= now:
            q = qs[i]
            tk = ctx.submit(gids[q["graph"]], tids[i], q["t"], q["seed"], 0, q["n"])
            pending[tk] = q["n"]
            i += 1
        for tk in list(pending):
            r = ctx.poll(tk, pending[tk])
            if r is not None:
                assert r["status"] == 0, r["status"]
                results.append(r)
                del pending[tk]
                if len(results) % 10 == 0:
                    print(f"[bench] serve {len(results)}/{nq} done", file=sys.stderr, flush=True)
        time.sleep(0.0005)
    stats = ctx.serve_stats()
    ctx.serve_stop()
    lat = np.array([r["done_s"] - r["submit_s"] for r in results])
    span = max(r["done_s"] for r in results) - min(r["submit_s"] for r in results)
    ncol = sum(q["n"] for q in qs)
    out = {"serving": {"queries": nq, "offered_qps": qps, "colorings": ncol,
                       "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
                       "colorings_per_s": round(ncol / span, 2), "queries_per_s": round(nq / span, 2),
                       "passes": int(stats["passes"]), "peak_table_GB": round(stats["peak_mem_bytes"] / 1e9, 1),
                       "streams": streams, "budget_GB": 200}}
    ctx.close()
    print(json.dumps(out), flush=True)


def gather_probe():
    """Ceiling of the DP's dominant access: whole passive rows gathered in a
    graph's neighbour order, from a table of one row per non-isolated vertex
    (rows relabelled by descending degree, as the library keeps them):
    RMAT scale 20 with rows of 126 sets x 8 colourings (1008 uint64, the
    widest step of the 10-vertex tree), and Chung-Lu n=4,194,304 with rows of
    462 sets x 2 colourings (924 uint64, the step (11,5,6) of the 12-vertex
    tree).  torch.index_select into a reused 32768-row buffer; GB/s counts the
    gathered (read) bytes only, so it is a lower bound of the read ceiling."""
    import numpy as np
    import torch
    from paper_1903_04395_amd import inputs as I
    out = {}
    for name, gen, W in (("rmat20", lambda: I.rmat(20, 16, seed=0), 1008),
                         ("chunglu4m", lambda: I.chung_lu(4194304, 30, 2.1, seed=3), 924)):
        g = gen()
        deg = g.degrees()
        order = np.argsort(-deg, kind="stable")
        rows = int((deg > 0).sum())
        new_id = np.empty(g.n, np.int64)
        new_id[order] = np.arange(g.n)
        idx = torch.from_numpy(new_id[g.col_idx.astype(np.int64)]).cuda()
        del g
        table = torch.ones((rows, W), dtype=torch.int64, device="cuda")
        chunk = 32768
        buf = torch.empty((chunk, W), dtype=torch.int64, device="cuda")

        def run():
            for c0 in range(0, idx.numel(), chunk):
                sel = idx[c0:c0 + chunk]
                torch.index_select(table, 0, sel, out=buf[:sel.numel()])
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        gathered = idx.numel() * W * 8
        out[name] = {"rows": rows, "row_bytes": W * 8, "gathers": int(idx.numel()), "ms": round(ms, 2),
                     "read_GBps": round(gathered / (ms / 1e3) / 1e9, 1)}
        print(f"[bench] gather probe {name}: {out[name]}", file=sys.stderr, flush=True)
        del table, buf, idx
        torch.cuda.empty_cache()
    # streaming references: a 4 GiB device copy (read + write) and a 16 GiB sum (read)
    a = torch.ones(1 << 29, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    big = torch.ones(1 << 31, dtype=torch.int64, device="cuda")
    for _ in range(2):
        b.copy_(a)
        big.sum()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    b.copy_(a)
    e[1].record()
    big.sum()
    e[2].record()
    torch.cuda.synchronize()
    out["stream"] = {"copy_GBps": round(2 * a.numel() * 8 / (e[0].elapsed_time(e[1]) / 1e3) / 1e9, 1),
                     "read_GBps": round(big.numel() * 8 / (e[1].elapsed_time(e[2]) / 1e3) / 1e9, 1)}
    print(f"[bench] stream: {out['stream']}", file=sys.stderr, flush=True)
    print(json.dumps({"gather_probe": out}), flush=True)


def configs_bench(only=None, tune_ok=True):
    """Per-configuration timings after a warm-up pass (allocation excluded):
    ER 2000 / P5 / k=5 (one colouring per call: launch latency); Chung-Lu
    n=4,194,304 (mean degree 30, exponent 2.1) / 12-vertex tree and 12-star /
    k=12 / 16 colourings; RMAT scale 19 / 15-vertex tree / k=15 / 4 colourings;
    RMAT scale 20 / 10-vertex tree / k=10 / 8 colourings (5 timed calls).
    The multi-colouring cases are timed with the planner's default knobs, then
    again after the autotuner picks the interleave and LDS limit."""
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    ctx = sc.Context(0)
    out = {}
    # (name, graph, templates, k, colourings per call, timed calls, autotune)
    cases = [("er2000-p5-k5", lambda: I.erdos_renyi(2000, 10000, seed=1), [("p5", 5, I.path(5), 0)], 5, 1, 200, False),
             ("chunglu4m-k12", lambda: I.chung_lu(4194304, 30, 2.1, seed=3),
              [("tree12", 12, I.prufer_tree(12, 3), -1), ("star12", 12, I.star(12), 0)], 12, 16, 1, True),
             ("rmat19-tree15-k15", lambda: I.rmat(19, 16, seed=4), [("tree15", 15, I.prufer_tree(15, 4), -1)],
              15, 4, 1, True),
             ("rmat20-tree10-k10", lambda: I.rmat(20, 16, seed=0), [("tree10", 10, I.prufer_tree(10, 0), -1)],
              10, 8, 5, True)]

    def timed_calls(gid, tid, R, reps):
        ctx.run(gid, tid, 0, R)                           # warm (allocation, tables)
        ctx.profile(True)
        t0 = time.perf_counter()
        for i in range(reps):
            ctx.run(gid, tid, R * (i + 1), R)
        dt = (time.perf_counter() - t0) / reps
        ctx.profile(False)
        steps = {}
        for r in ctx.profile_launches():
            if r["step"] >= 0:
                key = f"{r['step']}:{r['family']}:({r['h']},{r['a']},{r['p']})"
                steps[key] = steps.get(key, 0.0) + r["ms"] / reps
        return dt, ctx.profile_read(), {k: round(v, 2) for k, v in steps.items()}

    for gname, gen, tmpls, k, R, reps, tune in cases:
        if only and gname != only:
            continue
        tune = tune and tune_ok
        tg = time.time()
        g = gen()
        gid = ctx.load_graph(g)
        print(f"[bench] configs {gname}: n={g.n} nnz={g.nnz} ({time.time() - tg:.0f}s)", file=sys.stderr, flush=True)
        for tname, t, edges, root in tmpls:
            tid = ctx.load_template(t, edges, root)
            ctx.set_colors(k, 7)
            info0 = ctx.plan_info(gid, tid, R)
            dt0, fams, steps = timed_calls(gid, tid, R, reps)
            tuned, dt, info = None, dt0, info0
            if tune:
                tuned = ctx.autotune(gid, tid, R)
                info = ctx.plan_info(gid, tid, R)
                dt, fams, steps = timed_calls(gid, tid, R, reps)
            key = f"{gname}/{tname}"
            out[key] = {"colorings": R, "batch": info.batch, "interleave": info.interleave,
                        "passes": -(-R // info.batch), "tables_GB_per_pass": round(info.arena_bytes / 1e9, 1),
                        "s_per_call": round(dt, 4), "colorings_per_s": round(R / dt, 2),
                        "default_s_per_call": round(dt0, 4), "default_interleave": info0.interleave,
                        "autotuned": tuned,
                        "families_ms_per_call": {f: round(v["total_ms"] / reps, 2) for f, v in fams.items()},
                        "steps_ms_per_call": steps}
            print(f"[bench] configs {key}: {out[key]}", file=sys.stderr, flush=True)
        ctx.unload_graph(gid)
        del g
    ctx.close()
    print(json.dumps({"configs": out}), flush=True)


def exact_bench():
    """Exact wide counts beside the uint64 pass, per call after a warm-up:
    RMAT scale 20 / 10-vertex tree / k=10 / 8 colourings, and Chung-Lu
    n=4,194,304 / 12-star / k=12 / 16 colourings.  Every colouring of these
    workloads overflows 2^64: for the tree sc_run_exact adds residue passes,
    the star (one chain from its centre) takes one multi-limb pass; the star's
    residue route (chains off) is timed beside it."""
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    ctx = sc.Context(0)
    out = {}
    cases = [("rmat20-tree10-k10", lambda: I.rmat(20, 16, seed=0), 10, I.prufer_tree(10, 0), 0, 10, 1, 8),
             ("chunglu4m-star12-k12", lambda: I.chung_lu(4194304, 30, 2.1, seed=3), 12, I.star(12), 0, 12, 7, 16)]
    for name, gen, t, edges, root, k, seed, R in cases:
        g = gen()
        gid = ctx.load_graph(g)
        tid = ctx.load_template(t, edges, root)
        ctx.set_colors(k, seed)
        ctx.run(gid, tid, 0, R)
        ctx.run_exact(gid, tid, 0, R)
        t0 = time.perf_counter()
        c64, ovf, _, _ = ctx.run(gid, tid, R, R)
        t1 = time.perf_counter()
        counts, exact, hom, maps, copies = ctx.run_exact(gid, tid, R, R)
        t2 = time.perf_counter()
        t3 = time.perf_counter()
        hom2 = ctx.hom_count(gid, tid)
        t4 = time.perf_counter()
        out[name] = {"colorings": R, "overflowed": int(ovf.sum()), "exact": int(exact.sum()),
                     "s_uint64": round(t1 - t0, 4), "s_exact": round(t2 - t1, 4),
                     "exact_over_uint64": round((t2 - t1) / (t1 - t0), 2), "s_hom_count": round(t4 - t3, 4),
                     "hom_bound_log2": round(math.log2(hom2), 1) if hom2 > 0 else None,
                     "max_count_log2": round(math.log2(max(counts)), 1) if max(counts) > 0 else None,
                     "est_maps": maps, "est_copies": copies}
        if name.startswith("chunglu"):
            ctx.set_option(sc.SC_OPT_CHAIN, 0)
            ctx.run_exact(gid, tid, 0, R)
            t5 = time.perf_counter()
            c_res, e_res, _, _, _ = ctx.run_exact(gid, tid, R, R)
            t6 = time.perf_counter()
            ctx.set_option(sc.SC_OPT_CHAIN, sc.OPTION_DEFAULTS[sc.SC_OPT_CHAIN])
            assert list(c_res) == list(counts) and e_res.all()
            out[name]["s_exact_residue_route"] = round(t6 - t5, 4)
        print(f"[bench] exact {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.unload_graph(gid)
        del g
    ctx.close()
    print(json.dumps({"exact": out}), flush=True)


def ablation_bench():
    """The paper's pruning ablation (Sec. 7.1), on MI355X: per colouring, the
    FASCIA baseline (Algorithm 1: every split re-sums the passive column over
    the neighbours), PFASCIA (pruned: neighbour sums once), and the library's
    path (one colouring per pass, and 8 folded into a pass), on RMAT scale 16
    with seeded Pruefer trees of 6..10 vertices, k = t.  All four give the same
    counts (checked here)."""
    import numpy as np
    import torch
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    ctx = sc.Context(0)
    g = I.rmat(16, 16, seed=6)
    gid = ctx.load_graph(g)
    print(f"[bench] ablation graph n={g.n} nnz={g.nnz}", file=sys.stderr, flush=True)
    out = {}

    def clock(fn):
        fn()                                          # warm (allocation, tables)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    for t in range(6, 11):
        tid = ctx.load_template(t, I.prufer_tree(t, t))
        ctx.set_colors(t, 11)
        tf, (cf, _) = clock(lambda: ctx.run_ablation(gid, tid, sc.SC_ABL_FASCIA, 0, 1))
        tp, (cp, _) = clock(lambda: ctx.run_ablation(gid, tid, sc.SC_ABL_PFASCIA, 0, 1))
        t1, (c1, _, _, _) = clock(lambda: ctx.run(gid, tid, 0, 1))
        t8, (c8, _, _, _) = clock(lambda: ctx.run(gid, tid, 0, 8))
        assert int(cf[0]) == int(cp[0]) == int(c1[0]) == int(c8[0])
        out[f"tree{t}"] = {"fascia_ms": round(tf * 1e3, 2), "pfascia_ms": round(tp * 1e3, 2),
                           "libsc_1_ms": round(t1 * 1e3, 3), "libsc_8_ms_per_colouring": round(t8 * 1e3 / 8, 3),
                           "pruning_speedup": round(tf / tp, 2), "libsc_over_pfascia": round(tp / t1, 1)}
        print(f"[bench] ablation tree{t}: {out[f'tree{t}']}", file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps({"ablation": out}), flush=True)


def copy_probe():
    import torch
    a = torch.empty(1 << 27, dtype=torch.int64, device="cuda")   # 1 GiB
    a.fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 1 << 30, "copies": 3}), flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "exact.h"):
        with open(os.path.join(ROOT, "paper_1903_04395_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_step():
    """HBM bytes per DP step (all dp_ kernels of a pass over its steps) from the
    committed rocprofv3 counter summary, if it was taken from the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_step")


# the workload: (name, n, mean degree, exponent, graph seed), k, colouring seed,
# colourings per template per step, and the templates (name, t, edges, root)
CL = ("Chung-Lu", 4194304, 30, 2.1, 3)
K, SEED, R_STEP = 12, 7, 16


def templates():
    from paper_1903_04395_amd import inputs as I
    return [("tree12", 12, I.prufer_tree(12, 3), -1), ("star12", 12, I.star(12), 0)]


def host_info():
    """CPU model, logical cores and RAM of this host (for the CPU baseline)."""
    model, ram = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "ram_GiB": ram, "cpus_visible": os.cpu_count()}


def passes_of(launches):
    """Splits a launch trace into passes (each starts by clearing its result words)."""
    out = []
    for r in launches:
        if r["family"] == "zero" or not out:
            out.append([])
        out[-1].append(r)
    return out


def step_table(launches, sequence, rows, valu):
    """Per template and DP step (a chain of single-vertex attaches counts as one
    step): ms per step of the benchmark, the paper-layout compulsory bytes,
    the rooted-layout bytes, the multiply-adds executed, and the fraction of
    each roof; `bound` is the roof with the larger lower bound on the time.
    `sequence` names the template of each traced pass in order."""
    table = {}
    passes = passes_of(launches)
    if len(passes) != len(sequence):
        return None
    for name, ps in zip(sequence, passes):
        for r in ps:
            if r["step"] < 0:
                continue
            key = (name, r["step"])
            fam = r["family"]
            e = table.setdefault(key, {"template": name, "step": r["step"], "hap": None, "chain": False,
                                       "ms": 0.0, "alg_bytes": 0.0, "layout_bytes": 0.0, "mul_adds": 0.0,
                                       "colorings": 0})
            e["ms"] += r["ms"]
            e["alg_bytes"] += r["alg_bytes"]
            e["layout_bytes"] += r["layout_bytes"]
            if fam in ("row_gather", "row_hist", "chain"):
                h, a, p = r["h"], r["a"], r["p"]
                e["hap"] = [h, a, p]
                e["chain"] = fam == "chain"
                e["colorings"] += r["colorings"]
                # executed multiply-adds of the rooted-colour layout (a >= 2);
                # a chain runs the steps (a+1, a, 1) .. (h, h-1, 1)
                hs = [(hh, hh - 1) for hh in range(a + 1, h + 1)] if fam == "chain" else [(h, a)]
                for hh, aa in hs:
                    if aa > 1:
                        e["mul_adds"] += rows * math.comb(K - 1, hh - 1) * math.comb(hh - 1, aa - 1) * r["colorings"]
    out = []
    for e in sorted(table.values(), key=lambda x: (x["template"], x["step"])):
        if e["hap"] is None or not e["colorings"]:
            continue
        h, a, p = e["hap"]
        reps = e["colorings"] / R_STEP
        ms = e["ms"] / reps
        ab, lb, ma = e["alg_bytes"] / reps, e["layout_bytes"] / reps, e["mul_adds"] / reps
        form = 2 if p == 1 else (1 if math.comb(h - 1, a - 1) >= 32 else 0)
        t_hbm = ab / (PEAK_HBM_GBS * 1e9)
        t_alu = ma / valu[form] if ma else 0.0
        out.append({"template": e["template"], "step": e["step"], "hap": e["hap"], "chain": e["chain"],
                    "ms": round(ms, 3), "alg_GB": round(ab / 1e9, 2), "layout_GB": round(lb / 1e9, 2),
                    "G_mul_adds": round(ma / 1e9, 2),
                    "hbm_frac": round(t_hbm / (ms / 1e3), 3), "layout_hbm_frac": round(lb / 8e12 / (ms / 1e3), 3),
                    "valu_frac": round(t_alu / (ms / 1e3), 3) if ma else None,
                    "bound": "valu" if t_alu > t_hbm else "hbm"})
    return out


def golden_check(counts):
    """The colourings 0..15 of both templates against the oracle's residues and
    flags stored in tests/golden/full_size.json (written by a script that
    calls only the oracle), where the file holds them."""
    path = os.path.join(ROOT, "tests", "golden", "full_size.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    out = {}
    for name, key in (("tree12", "chunglu4m_tree12_k12"), ("star12", "chunglu4m_star12_k12")):
        e = data.get(key)
        if not e or e.get("seed") != SEED or e.get("k") != K or name not in counts:
            continue
        c, f = counts[name]
        hits = [r for r in e["results"] if int(r) < len(c)]
        ok = all(int(c[int(r)]) == int(e["results"][r][0]) and int(f[int(r)]) == int(e["results"][r][1])
                 for r in hits)
        out[name] = {"colorings": len(hits), "equal": ok}
    return out


def extras(ctx, gid3, star_tid):
    """Side measurements for the same line, after the timed region: exact
    counts (sc_run_exact: one multi-limb pass, the star being one chain from its
    centre) of 16 colourings of the Chung-Lu 12-star beside its uint64 pass; then, on RMAT scale 20 / 10-vertex
    Pruefer tree (seed 0) / k = 10, the uint64 pass of 8 colourings, exact
    counts of 8 colourings, and the plain per-colouring launch loop (one
    colouring per sc_run) against the batched form (8 colourings folded into a
    pass, replayed from a captured hipGraph) on 16 colourings."""
    import numpy as np
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc
    out = {}
    ctx.set_colors(K, SEED)
    ctx.run_exact(gid3, star_tid, 0, R_STEP)                  # warm
    t0 = time.perf_counter()
    ctx.run(gid3, star_tid, R_STEP, R_STEP)
    t1 = time.perf_counter()
    _, exact, _, _, _ = ctx.run_exact(gid3, star_tid, R_STEP, R_STEP)
    t2 = time.perf_counter()
    out["chunglu4m_star12_exact"] = {"colorings": R_STEP, "certified": int(exact.sum()),
                                     "s_uint64": round(t1 - t0, 3), "s_exact": round(t2 - t1, 3),
                                     "exact_colorings_per_s": round(R_STEP / (t2 - t1), 2),
                                     "exact_over_uint64": round((t2 - t1) / (t1 - t0), 2)}
    print(f"[bench] extras: {out}", file=sys.stderr, flush=True)
    ctx.unload_graph(gid3)
    g = I.rmat(20, 16, seed=0)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(10, I.prufer_tree(10, 0))
    ctx.set_colors(10, 1)
    info = ctx.plan_info(gid, tid, 8)
    ctx.run(gid, tid, 0, 8)
    reps = 5
    t0 = time.perf_counter()
    for i in range(reps):
        ctx.run(gid, tid, 8 * (i + 1), 8)
    dt = (time.perf_counter() - t0) / reps
    ctx.run_exact(gid, tid, 0, 8)
    t1 = time.perf_counter()
    _, exact, _, _, _ = ctx.run_exact(gid, tid, 8, 8)
    dte = time.perf_counter() - t1
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 1)
    ctx.run(gid, tid, 0, 1)
    t0 = time.perf_counter()
    plain = [ctx.run(gid, tid, r, 1)[0][0] for r in range(16)]
    dt_p = time.perf_counter() - t0
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 8)
    ctx.set_option(sc.SC_OPT_GRAPH, 1)
    ctx.run(gid, tid, 0, 16)
    t0 = time.perf_counter()
    batched = ctx.run(gid, tid, 0, 16)[0]
    dt_b = time.perf_counter() - t0
    ctx.set_option(sc.SC_OPT_GRAPH, 0)
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 64)
    assert np.array_equal(np.asarray(plain, np.uint64), batched)
    out["rmat20_tree10_k10_b8"] = {
        "ms_per_pass": round(dt * 1e3, 2), "colorings_per_s": round(8 / dt, 1),
        "G_updates_per_s": round(8 * (info.spmm_updates + info.ema_updates) / dt / 1e9, 1),
        "exact_ms_per_8": round(dte * 1e3, 1), "exact_certified": int(exact.sum()),
        "plain_colorings_per_s": round(16 / dt_p, 1), "batched_colorings_per_s": round(16 / dt_b, 1),
        "batched_over_plain": round(dt_p / dt_b, 2)}
    print(f"[bench] extras: {out['rmat20_tree10_k10_b8']}", file=sys.stderr, flush=True)
    ctx.unload_graph(gid)
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gather_probe:
        gather_probe()
        return
    if args.forms or args.serve or args.configs or args.exact or args.ablation:
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        if args.forms:
            forms_bench()
        elif args.serve:
            serve_bench(args.queries, args.qps, args.streams)
        elif args.exact:
            exact_bench()
        elif args.ablation:
            ablation_bench()
        else:
            configs_bench(args.only, not args.no_tune)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); splitting the colourings "
              "across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1903_04395_amd import inputs as I
    from paper_1903_04395_amd import sc

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t_gen = time.time()
    _, n0, deg, gamma, gseed = CL
    g = I.chung_lu(n0, deg, gamma, seed=gseed)
    print(f"[bench] graph n={g.n} nnz={g.nnz} generated in {time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)

    ctx = sc.Context(0)
    for o in args.opt:
        key, val = o.split("=")
        ctx.set_option(int(key), int(val))
    gid = ctx.load_graph(g)
    ctx.set_colors(K, SEED)
    tmpls, infos, plans, tuned = {}, {}, {}, {}
    upd = 0.0
    for name, t, edges, root in templates():
        tmpls[name] = ctx.load_template(t, edges, root)
    if args.tune_load:
        print(f"[bench] loaded {ctx.tune_load(args.tune_load)} tuning entries", file=sys.stderr, flush=True)
    for name, tid in tmpls.items():
        if not args.no_autotune and not args.tune_load:   # untimed: the autotuner's real passes
            tt = time.time()
            tuned[name] = ctx.autotune(gid, tid, R_STEP)
            print(f"[bench] {name}: autotuned {tuned[name]} in {time.time() - tt:.0f}s", file=sys.stderr, flush=True)
        info = ctx.plan_info(gid, tid, R_STEP)
        infos[name], plans[name] = info, info.steps()
    if args.tune_save:
        ctx.tune_save(args.tune_save)
    for name, info in infos.items():
        upd += (info.spmm_updates + info.ema_updates) * R_STEP
        print(f"[bench] {name}: root={info.root} steps={info.steps()} batch={info.batch} "
              f"interleave={info.interleave} arena={info.arena_bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)

    def step(first):
        res = {}
        for name, tid in tmpls.items():
            c, f, _, _ = ctx.run(gid, tid, first, R_STEP)
            res[name] = (c, f)
        return res

    first = 0
    golden = None
    for w in range(max(args.warmup, 1)):             # colourings 0..15 first: the golden check
        res = step(first)
        if w == 0:
            golden = golden_check(res)
        first += R_STEP
        print(f"[bench] warm-up step {w + 1} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(first)
        first += R_STEP
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    fams = ctx.profile_read()
    launches = ctx.profile_launches()
    print(f"[bench] {args.steps} timed steps in {elapsed:.2f}s", file=sys.stderr, flush=True)

    colorings = args.steps * R_STEP * len(tmpls)
    value = args.steps * upd / elapsed / 1e9
    dp_f = [f for f in ("split", "row_gather", "row_hist") if f in fams]
    dp_ms = sum(fams[f]["total_ms"] for f in dp_f)
    dp_alg = sum(fams[f]["alg_bytes"] for f in dp_f)
    dp_lay = sum(fams[f]["layout_bytes"] for f in dp_f)
    dp_launches = sum(fams[f]["launches"] for f in ("row_gather", "row_hist") if f in fams)
    achieved = dp_alg / (dp_ms / 1e3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_per_step(),
        "kernel": "DP step = dp_split_kernel (rows above the segment size) + dp_row_kernel (dp_root_kernel for "
                  "the root step (k, 1, k-1))",
        "bytes": "paper layout: binom(k, s) colour sets per row, every vertex; fused steps",
        "avg_step_ms": round(dp_ms / dp_launches, 4),
        "alg_bytes_per_step": dp_alg / dp_launches,
        "layout_achieved": round(dp_lay / (dp_ms / 1e3) / 1e9, 1),
        "layout_frac": round(dp_lay / (dp_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
        "layout_bytes_per_step": dp_lay / dp_launches,
        "share_of_gpu_time": round(dp_ms / sum(f["total_ms"] for f in fams.values()), 3),
    }
    valu = {f: ctx.valu_probe(f) for f in (0, 1, 2)}
    rows = int((np.diff(g.row_ptr) > 0).sum())        # table rows: the non-isolated vertices
    sequence = []
    for _ in range(args.steps):
        for name in tmpls:
            sequence += [name] * -(-R_STEP // infos[name].batch)
    steps_tab = step_table(launches, sequence, rows, valu)
    out = {
        "metric": "SpMM+eMA G-updates/s & colorings/s (bit-exact); p50/p99 query latency",
        "value": round(value, 2), "unit": "G-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "colorings_per_s": round(colorings / elapsed, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "chunglu4m-k12-tree12+star12-r16",
                   "graph": f"Chung-Lu n={g.n}, mean degree {deg}, exponent {gamma}, seed {gseed}",
                   "n": g.n, "nnz": g.nnz, "k": K, "seed": SEED, "colorings_per_template_per_step": R_STEP,
                   "templates": {nm: {"template": "12-vertex Pruefer tree (seed 3)" if nm == "tree12" else "12-star",
                                      "root": infos[nm].root, "steps": infos[nm].steps(),
                                      "batch": infos[nm].batch, "interleave": infos[nm].interleave,
                                      "tables_GB_per_pass": round(infos[nm].arena_bytes / 1e9, 1),
                                      "autotuned": tuned.get(nm)}
                                 for nm in tmpls}},
        "roofline": roofline,
        "valu_mul_adds_per_s": {["128-bit", "3-multiply", "32-bit operand"][f]: v for f, v in valu.items()},
        "families_ms_per_step": {k: round(v["total_ms"] / args.steps, 2) for k, v in fams.items()},
        "steps_table": steps_tab,
        "golden_check": golden,
    }

    if not args.no_cpu_baseline:
        import oracle as O
        t4, e4 = 4, I.star(4)
        plan4 = O.root_plan(t4, e4, 0, "small")
        s4 = sc.sc_plan_template(t4, e4, 0, K, g.n, g.nnz, 1)
        sample = first - R_STEP
        tc = time.perf_counter()
        oc, of = O.count(g, t4, plan4, K, SEED, sample, 1)
        dt = time.perf_counter() - tc
        tid4 = ctx.load_template_plan(t4, plan4[0], plan4[1])
        gc, gf, _, _ = ctx.run(gid, tid4, sample, 1)
        out["cpu_baseline"] = {
            "value": round((s4.spmm_updates + s4.ema_updates) / dt / 1e9, 4), "unit": "G-updates/s",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"the first three DP steps of both templates' plans (the 4-vertex star rooted at its "
                      f"centre, k = {K}), colouring {sample}, on the whole graph; {dt:.1f} s",
            "host": host_info(),
        }
        out["parity_sample"] = {"coloring": int(sample), "template": "4-vertex star (the plans' first three steps)",
                                "gpu": [str(int(gc[0])), int(gf[0])], "oracle": [str(int(oc[0])), int(of[0])],
                                "equal": bool(int(gc[0]) == int(oc[0]) and int(gf[0]) == int(of[0]))}
    if not args.no_extras:
        out["extras"] = extras(ctx, gid, tmpls["star12"])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
