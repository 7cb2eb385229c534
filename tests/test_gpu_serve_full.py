"""The serving mix at full scale: three resident RMAT graphs (scale 18, 20,
22; 16 edges per vertex) and a sample of the seeded Poisson query stream
(random 3..12-vertex trees, k = t, 1..32 colourings).  Every query's
per-colouring residues and flags are identical when it runs alone (sc_run)
and inside the serving loop's continuous batching (200 GB table budget, four
streams, queries submitted at their arrival times); queries of at most six
vertices are also checked against the CPU oracle on their first colourings."""
import time

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc

pytestmark = pytest.mark.gpu

SCALES = (18, 20, 22)
N_QUERIES = 14


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    ctx = sc.Context(0)
    graphs, gids = [], []
    for scale in SCALES:
        t0 = time.time()
        g = I.rmat(scale, 16, seed=scale)
        graphs.append(g)
        gids.append(ctx.load_graph(g))
        print(f"[case] serving graph scale {scale}: n={g.n} nnz={g.nnz} ({time.time() - t0:.0f}s)", flush=True)
    yield ctx, graphs, gids
    ctx.close()


def test_serving_mix_full_scale_alone_equals_mixed(setup):
    ctx, graphs, gids = setup
    qs = I.serving_queries(N_QUERIES, qps=200.0, seed=2019)
    tids = [ctx.load_template(q["t"], q["edges"]) for q in qs]
    alone = []
    for i, q in enumerate(qs):
        ctx.set_colors(q["t"], q["seed"])
        t0 = time.perf_counter()
        c, f, _, _ = ctx.run(gids[q["graph"]], tids[i], 0, q["n"])
        print(f"[case] alone {i}: scale {SCALES[q['graph']]} t={q['t']} colourings {q['n']} "
              f"({time.perf_counter() - t0:.2f}s)", flush=True)
        alone.append((c.copy(), f.copy()))
    ctx.serve_start(mem_budget_bytes=200 * 10**9, max_inflight=4, max_batch=64)
    try:
        pending, mixed = {}, {}
        t0 = time.perf_counter()
        i = 0
        while i < len(qs) or pending:
            now = time.perf_counter() - t0
            while i < len(qs) and qs[i]["at"] <= now:
                q = qs[i]
                pending[ctx.submit(gids[q["graph"]], tids[i], q["t"], q["seed"], 0, q["n"])] = i
                i += 1
            for tk in list(pending):
                r = ctx.poll(tk, qs[pending[tk]]["n"])
                if r is not None:
                    assert r["status"] == 0, r
                    mixed[pending.pop(tk)] = r
            time.sleep(0.0005)
        stats = ctx.serve_stats()
    finally:
        ctx.serve_stop()
    print(f"[case] mixed: {len(mixed)} queries in {stats['passes']} passes, "
          f"peak tables {stats['peak_mem_bytes'] / 1e9:.1f} GB", flush=True)
    for i, q in enumerate(qs):
        assert np.array_equal(mixed[i]["counts"], alone[i][0]), i
        assert np.array_equal(mixed[i]["overflow"], alone[i][1]), i
    checked = 0
    for i, q in enumerate(qs):
        if q["t"] > 6:
            continue
        ctx.set_colors(q["t"], q["seed"])
        info = ctx.plan_info(gids[q["graph"]], tids[i], q["n"])
        R = min(q["n"], 2)
        oc, of = O.count(graphs[q["graph"]], q["t"], (info.root, info.children()), q["t"], q["seed"], 0, R)
        print(f"[case] oracle {i}: scale {SCALES[q['graph']]} t={q['t']}", flush=True)
        assert np.array_equal(alone[i][0][:R], oc) and np.array_equal(alone[i][1][:R], of), i
        checked += 1
    assert checked >= 3
