"""Benchmark: colour-coding tree counting on one MI355X.

Workload (the headline configuration): RMAT scale 20 (1,048,576 vertices, 16
edges per vertex, a/b/c/d = .57/.19/.19/.05, symmetrised, deduplicated,
self-loops removed, labels permuted), a 10-vertex template tree from a seeded
Pruefer sequence, k = 10 colours, 8 colourings folded into one pass.  One
"step" is one sc_run over a fresh batch of 8 colourings (colouring, every DP
step, root reduction, 9-byte-per-colouring result copy); the graph is resident
in HBM before the timed region starts.

Prints one JSON line.  `value` is G-updates/s: per colouring the neighbour-sum
updates sum_steps nnz*C(k,p) plus the multiply-adds sum_steps n*C(k,h)*C(h,a)
(n*C(k,h) for a select step), over the timed wall time.  `roofline` describes
the kernel family with the largest share of time, from HIP events recorded by
libsc on its stream around every launch in the timed region.  `cpu_baseline`
times the CPU oracle on one colouring of the same workload (and checks that
colouring's residue and flag against the GPU).
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

# HIP kernel behind each libsc kernel family
KERNEL_OF = {
    "row_gather": "dp_row_kernel<false, *>", "row_hist": "dp_row_kernel<true, *>",
    "split": "dp_split_kernel<*>", "reduce": "reduce_kernel", "color": "color_kernel",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=20, help="RMAT scale (20 = the headline workload)")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--opt", action="append", default=[], help="libsc option NUM=VALUE (ablation)")
    ap.add_argument("--breakdown", action="store_true", help="also print the per-family table")
    ap.add_argument("--configs", action="store_true",
                    help="timings of the other configurations (ER 2000 / Chung-Lu 4M k=12 / RMAT-19 k=15)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="only time whole-row gathers of the widest step's rows in RMAT-20 neighbour order")
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
    call), on the same colourings; results must agree."""
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
        # batched: B colourings per pass, hipGraph replay
        ctx.set_option(sc.SC_OPT_MAX_BATCH, B)
        ctx.set_option(sc.SC_OPT_GRAPH, 1)
        ctx.run(gid, tid, 0, R)
        dt_b, (cb, _, _, _) = timed(lambda: ctx.run(gid, tid, 0, R))
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
        ctx.set_option(sc.SC_OPT_MAX_BATCH, 64)
        assert np.array_equal(np.asarray(plain, np.uint64), cb), name
        out[name] = {"colorings": R, "batch": B, "plain_colorings_per_s": round(R / dt_p, 1),
                     "batched_colorings_per_s": round(R / dt_b, 1), "ratio": round(dt_p / dt_b, 2)}
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
    rng = np.random.default_rng(2019)
    ctx = sc.Context(0)
    gids = []
    for scale in (18, 20, 22):
        tg = time.time()
        g = I.rmat(scale, 16, seed=scale)
        gids.append(ctx.load_graph(g))
        print(f"[bench] serve graph scale {scale}: n={g.n} nnz={g.nnz} ({time.time() - tg:.0f}s)",
              file=sys.stderr, flush=True)
        del g
    qs = []
    t_arr = 0.0
    for i in range(nq):
        t_arr += rng.exponential(1 / qps)
        t = int(rng.integers(3, 13))
        qs.append(dict(at=t_arr, graph=int(rng.integers(0, 3)), t=t, edges=I.prufer_tree(t, 10_000 + i),
                       n=int(rng.integers(1, 33)), seed=int(rng.integers(0, 1 << 40))))
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
    """Ceiling of the DP's dominant access: whole passive rows of the widest
    step (126 sets x 8 colourings = 1008 uint64, 8064 bytes) gathered in the
    neighbour order of RMAT scale 20, from a table of one row per non-isolated
    vertex (rows relabelled by descending degree, as the library keeps them).
    torch.index_select into a reused 32768-row buffer; GB/s counts the
    gathered (read) bytes only, so it is a lower bound of the read ceiling."""
    import numpy as np
    import torch
    from paper_1903_04395_amd import inputs as I
    g = I.rmat(20, 16, seed=0)
    deg = g.degrees()
    order = np.argsort(-deg, kind="stable")
    rows = int((deg > 0).sum())
    new_id = np.empty(g.n, np.int64)
    new_id[order] = np.arange(g.n)
    idx = torch.from_numpy(new_id[g.col_idx.astype(np.int64)]).cuda()
    W = 1008
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
    print(json.dumps({"gather_probe": {"rows": rows, "row_bytes": W * 8, "gathers": int(idx.numel()),
                                       "ms": round(ms, 2),
                                       "read_GBps": round(gathered / (ms / 1e3) / 1e9, 1)}}), flush=True)


def configs_bench():
    """Per-configuration timings after a warm-up pass (allocation excluded):
    ER 2000 / P5 / k=5 (one colouring per call: launch latency); Chung-Lu
    n=4,194,304 (mean degree 30, exponent 2.1) / 12-vertex tree and 12-star /
    k=12 / 16 colourings; RMAT scale 19 / 15-vertex tree / k=15 / 4 colourings.
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
              15, 4, 1, True)]

    def timed_calls(gid, tid, R, reps):
        ctx.run(gid, tid, 0, R)                           # warm (allocation, tables)
        ctx.profile(True)
        t0 = time.perf_counter()
        for i in range(reps):
            ctx.run(gid, tid, R * (i + 1), R)
        dt = (time.perf_counter() - t0) / reps
        ctx.profile(False)
        return dt, ctx.profile_read()

    for gname, gen, tmpls, k, R, reps, tune in cases:
        tg = time.time()
        g = gen()
        gid = ctx.load_graph(g)
        print(f"[bench] configs {gname}: n={g.n} nnz={g.nnz} ({time.time() - tg:.0f}s)", file=sys.stderr, flush=True)
        for tname, t, edges, root in tmpls:
            tid = ctx.load_template(t, edges, root)
            ctx.set_colors(k, 7)
            info0 = ctx.plan_info(gid, tid, R)
            dt0, fams = timed_calls(gid, tid, R, reps)
            tuned, dt, info = None, dt0, info0
            if tune:
                tuned = ctx.autotune(gid, tid, R)
                info = ctx.plan_info(gid, tid, R)
                dt, fams = timed_calls(gid, tid, R, reps)
            key = f"{gname}/{tname}"
            out[key] = {"colorings": R, "batch": info.batch, "interleave": info.interleave,
                        "passes": -(-R // info.batch), "tables_GB_per_pass": round(info.arena_bytes / 1e9, 1),
                        "s_per_call": round(dt, 4), "colorings_per_s": round(R / dt, 2),
                        "default_s_per_call": round(dt0, 4), "default_interleave": info0.interleave,
                        "autotuned": tuned,
                        "families_ms_per_call": {f: round(v["total_ms"] / reps, 2) for f, v in fams.items()}}
            print(f"[bench] configs {key}: {out[key]}", file=sys.stderr, flush=True)
        ctx.unload_graph(gid)
        del g
    ctx.close()
    print(json.dumps({"configs": out}), flush=True)


def exact_bench():
    """Exact wide counts beside the uint64 pass, per call after a warm-up:
    RMAT scale 20 / 10-vertex tree / k=10 / 8 colourings, and Chung-Lu
    n=4,194,304 / 12-star / k=12 / 16 colourings.  Every colouring of these
    workloads overflows 2^64, so sc_run_exact adds three residue passes."""
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
        print(f"[bench] exact {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.unload_graph(gid)
        del g
    ctx.close()
    print(json.dumps({"exact": out}), flush=True)


def ablation_bench():
    """The paper's pruning ablation (Sec. 6.3), on MI355X: per colouring, the
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
            configs_bench()
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
    g = I.rmat(args.scale, 16, seed=0)
    t, k, B, seed = 10, 10, args.batch, 1
    edges = I.prufer_tree(t, 0)
    print(f"[bench] graph n={g.n} nnz={g.nnz} generated in {time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)

    ctx = sc.Context(0)
    for o in args.opt:
        key, val = o.split("=")
        ctx.set_option(int(key), int(val))
    gid = ctx.load_graph(g)
    tid = ctx.load_template(t, edges)
    ctx.set_colors(k, seed)
    info = ctx.plan_info(gid, tid, B)
    upd_per_coloring = info.spmm_updates + info.ema_updates
    print(f"[bench] plan root={info.root} steps={info.steps()} modes={info.modes()} batch={info.batch} "
          f"arena={info.arena_bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)

    first = 0
    for _ in range(args.warmup):
        ctx.run(gid, tid, first, B)
        first += B
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, ovf, _, _ = ctx.run(gid, tid, first, B)
        first += B
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    fams = ctx.profile_read()
    last_first = first - B

    colorings = args.steps * B
    value = colorings * upd_per_coloring / elapsed / 1e9
    # the DP step: each row kernel launch with the split pre-pass before it
    dp_f = [f for f in ("split", "row_gather", "row_hist") if f in fams]
    dp = {"total_ms": sum(fams[f]["total_ms"] for f in dp_f),
          "alg_bytes": sum(fams[f]["alg_bytes"] for f in dp_f),
          "launches": sum(fams[f]["launches"] for f in ("row_gather", "row_hist") if f in fams)}
    achieved = dp["alg_bytes"] / (dp["total_ms"] / 1e3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_per_step(),
        "kernel": "DP step = dp_split_kernel (rows above the segment size) + dp_row_kernel",
        "avg_step_ms": round(dp["total_ms"] / dp["launches"], 4),
        "alg_bytes_per_step": dp["alg_bytes"] / dp["launches"],
        "share_of_gpu_time": round(dp["total_ms"] / sum(f["total_ms"] for f in fams.values()), 3),
    }
    # passive rows gathered per pass: nnz * C(k-1, p-1) words per colouring for
    # every step with p >= 2 (row kernels and the split pre-pass)
    gathered = sum(g.nnz * math.comb(k - 1, p - 1) * 8 * B for h, a, p in info.steps() if p > 1)
    gather_ms = sum(fams[f]["total_ms"] for f in ("row_gather", "split") if f in fams) / args.steps
    roofline["gathered_GBps"] = round(gathered / (gather_ms / 1e3) / 1e9, 1) if gather_ms else None
    out = {
        "metric": "SpMM+eMA G-updates/s & colorings/s (bit-exact); p50/p99 query latency",
        "value": round(value, 2), "unit": "G-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "colorings_per_s": round(colorings / elapsed, 2),
        "exec_updates_per_s": round(colorings * info.exec_updates / elapsed / 1e9, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}-tree10-k10-b{B}", "graph": f"RMAT scale {args.scale}, 16 edges/vertex",
                   "n": g.n, "nnz": g.nnz, "template": "10-vertex Pruefer tree (seed 0)", "k": k,
                   "colorings_per_step": B, "root": info.root, "steps": info.steps(),
                   "modes": info.modes()},
        "roofline": roofline,
        "families_ms_per_step": {k: round(v["total_ms"] / args.steps, 2) for k, v in fams.items()},
    }
    if args.breakdown:
        print(json.dumps({"breakdown": fams}), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        import oracle as O
        plan = (info.root, info.children())
        tc = time.perf_counter()
        oc, of = O.count(g, t, plan, k, seed, last_first, 1)
        dt = time.perf_counter() - tc
        out["cpu_baseline"] = {
            "value": round(upd_per_coloring / dt / 1e9, 4), "unit": "G-updates/s",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"1 colouring (index {last_first}) of the same workload, whole graph; {dt:.1f} s",
        }
        out["parity_sample"] = {"coloring": int(last_first),
                                "gpu": [str(int(counts[0])), int(ovf[0])],
                                "oracle": [str(int(oc[0])), int(of[0])],
                                "equal": bool(int(counts[0]) == int(oc[0]) and int(ovf[0]) == int(of[0]))}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
