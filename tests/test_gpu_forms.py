"""GPU tests of the batched form (sc_run_batch), hipGraph replay, the
autotuner and the serving loop: every result is checked against the CPU
oracle or against the plain sc_run path (itself oracle-checked), bit-exact on
(residue, overflow flag)."""
import math
import time

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = sc.Context(0)
    yield c
    c.close()


def oracle_for(ctx, g, gid, tid, t, k, seed, first, n):
    ctx.set_colors(k, seed)
    info = ctx.plan_info(gid, tid, n)
    return O.count(g, t, (info.root, info.children()), k, seed, first, n)


TEMPLATES = [(5, I.path(5), 5), (8, I.prufer_tree(8, 1), 8), (6, I.star(6), 7), (10, I.prufer_tree(10, 4), 10),
             (3, I.path(3), 3)]


def test_batch_of_mixed_templates_matches_oracle(ctx):
    g = I.rmat(12, 16, seed=31)
    gid = ctx.load_graph(g)
    tids = [ctx.load_template(t, e) for t, e, _ in TEMPLATES]
    jobs = []
    for i, ((t, e, k), tid) in enumerate(zip(TEMPLATES, tids)):
        jobs.append({"graph_id": gid, "tmpl_id": tid, "k": k, "seed": 100 + i, "first": 3 * i, "n": 5 + 4 * i})
    say("batch of", len(jobs), "jobs")
    out = ctx.run_batch(jobs)
    for (t, e, k), j, (cnt, ovf, em, ec, st) in zip(TEMPLATES, jobs, out):
        assert st == 0
        oc, of = oracle_for(ctx, g, gid, j["tmpl_id"], t, k, j["seed"], j["first"], j["n"])
        assert np.array_equal(cnt, oc) and np.array_equal(ovf, of)
        om, oco = O.estimate(oc, of, k, t, O.aut(t, e))
        assert (math.isnan(em) and math.isnan(om)) or em == pytest.approx(om, rel=1e-12)
    ctx.unload_graph(gid)


def test_batch_reports_bad_jobs_and_runs_the_rest(ctx):
    g = I.erdos_renyi(500, 2000, 3)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(4, I.path(4))
    jobs = [{"graph_id": gid, "tmpl_id": tid, "k": 3, "seed": 1, "n": 2},          # k < t
            {"graph_id": gid, "tmpl_id": tid, "k": 4, "seed": 1, "n": 6},
            {"graph_id": gid + 77, "tmpl_id": tid, "k": 4, "seed": 1, "n": 2}]    # unknown graph
    out = ctx.run_batch(jobs)
    assert out[0][4] == sc.SC_EINVAL and out[2][4] == sc.SC_ENOTFOUND and out[1][4] == 0
    oc, of = oracle_for(ctx, g, gid, tid, 4, 4, 1, 0, 6)
    assert np.array_equal(out[1][0], oc) and np.array_equal(out[1][1], of)
    ctx.unload_graph(gid)


def test_graph_replay_matches_eager(ctx):
    """Each pass replays a captured hipGraph; replays run with eager work and
    synchronisations between them, and every replay is checked."""
    g = I.rmat(12, 16, seed=32)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(9, I.prufer_tree(9, 32))
    ctx.set_colors(9, 77)
    eager = [ctx.run(gid, tid, 8 * i, 8)[:2] for i in range(4)]
    ctx.set_option(sc.SC_OPT_GRAPH, 1)
    try:
        for rep in range(3):
            for i in range(4):
                say("replay", rep, i)
                c, f, _, _ = ctx.run(gid, tid, 8 * i, 8)
                assert np.array_equal(c, eager[i][0]) and np.array_equal(f, eager[i][1])
                ctx.set_option(sc.SC_OPT_GRAPH, 0)              # eager work between replays
                c2, f2, _, _ = ctx.run(gid, tid, 8 * i + 3, 5)
                ctx.set_option(sc.SC_OPT_GRAPH, 1)
                oc, of = oracle_for(ctx, g, gid, tid, 9, 9, 77, 8 * i + 3, 5)
                assert np.array_equal(c2, oc) and np.array_equal(f2, of)
        # a batch through replays as well
        out = ctx.run_batch([{"graph_id": gid, "tmpl_id": tid, "k": 9, "seed": 77, "first": 8 * i, "n": 8}
                             for i in range(4)])
        for i in range(4):
            assert np.array_equal(out[i][0], eager[i][0]) and np.array_equal(out[i][1], eager[i][1])
    finally:
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
    ctx.unload_graph(gid)


def test_whole_call_graph_matches_eager_and_oracle(ctx):
    """SC_OPT_GRAPH = 2: every pass of a call -- jobs on two graphs, templates
    of 3 to 10 vertices, k from 3 to 10, several passes per job -- is captured
    into one hipGraph and replayed with one launch.  The replays run with
    eager calls and synchronisations between them; each is checked against
    the eager results, which are checked against the oracle."""
    g1 = I.rmat(12, 16, seed=33)
    g2 = I.erdos_renyi(3000, 12000, 34)
    gids = [ctx.load_graph(g1), ctx.load_graph(g2)]
    tids = [ctx.load_template(t, e) for t, e, _ in TEMPLATES]
    jobs = []
    for i, ((t, e, k), tid) in enumerate(zip(TEMPLATES, tids)):
        for gi in range(2):
            jobs.append({"graph_id": gids[gi], "tmpl_id": tid, "k": k, "seed": 500 + 7 * i + gi,
                         "first": 2 * i, "n": 6 + 3 * i})
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 4)                       # several passes per job
    try:
        eager = ctx.run_batch(jobs)
        for j, (cnt, ovf, _, _, st) in zip(jobs, eager):
            assert st == 0
            i = tids.index(j["tmpl_id"])
            t, _, k = TEMPLATES[i]
            g = g1 if j["graph_id"] == gids[0] else g2
            oc, of = oracle_for(ctx, g, j["graph_id"], j["tmpl_id"], t, k, j["seed"], j["first"], j["n"])
            assert np.array_equal(cnt, oc) and np.array_equal(ovf, of)
        ctx.set_option(sc.SC_OPT_GRAPH, 2)
        for rep in range(3):
            say("whole-call replay", rep)
            out = ctx.run_batch(jobs)
            for (cnt, ovf, em, ec, st), (ecnt, eovf, eem, eec, _) in zip(out, eager):
                assert st == 0 and np.array_equal(cnt, ecnt) and np.array_equal(ovf, eovf)
                assert (math.isnan(em) and math.isnan(eem)) or em == eem
            ctx.set_option(sc.SC_OPT_GRAPH, 0)                   # eager work between replays
            ctx.set_colors(TEMPLATES[1][2], 9)
            c2, f2, _, _ = ctx.run(gids[0], tids[1], 40 + rep, 3)
            ctx.set_option(sc.SC_OPT_GRAPH, 2)
            oc, of = oracle_for(ctx, g1, gids[0], tids[1], TEMPLATES[1][0], TEMPLATES[1][2], 9, 40 + rep, 3)
            assert np.array_equal(c2, oc) and np.array_equal(f2, of)
        # other seeds and colouring ranges replay the same graph (same call shape)
        moved = [dict(j, seed=j["seed"] + 1000, first=j["first"] + 17) for j in jobs]
        out = ctx.run_batch(moved)
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
        ref = ctx.run_batch(moved)
        for (cnt, ovf, _, _, st), (rcnt, rovf, _, _, _) in zip(out, ref):
            assert st == 0 and np.array_equal(cnt, rcnt) and np.array_equal(ovf, rovf)
        # a single sc_run of several passes through the whole-call graph
        ctx.set_option(sc.SC_OPT_GRAPH, 2)
        ctx.set_colors(9, 3)
        t9 = ctx.load_template(9, I.prufer_tree(9, 35))
        for rep in range(2):
            c, f, _, _ = ctx.run(gids[0], t9, 5, 11)
            ctx.set_option(sc.SC_OPT_GRAPH, 0)
            ce, fe, _, _ = ctx.run(gids[0], t9, 5, 11)
            ctx.set_option(sc.SC_OPT_GRAPH, 2)
            assert np.array_equal(c, ce) and np.array_equal(f, fe)
    finally:
        ctx.set_option(sc.SC_OPT_GRAPH, 0)
        ctx.set_option(sc.SC_OPT_MAX_BATCH, 64)
    for gid in gids:
        ctx.unload_graph(gid)
    for bad in (-1, 3):
        with pytest.raises(sc.ScError):
            ctx.set_option(sc.SC_OPT_GRAPH, bad)


def test_autotune_keeps_results_and_round_trips(ctx, tmp_path):
    g = I.rmat(13, 16, seed=33)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(10, I.prufer_tree(10, 33))
    ctx.set_colors(10, 5)
    before = ctx.run(gid, tid, 0, 8)[:2]
    tune = ctx.autotune(gid, tid, 8)
    say("tuned", tune)
    assert tune["batch"] == 8 and tune["trials"] == 16 + 3 + 2
    assert tune["interleave"] in (1, 2, 4, 8) and tune["lds_max"] in (32768, 65536, 98304, 131072)
    assert tune["seg"] in (256, 512, 1024, 2048) and tune["wave_row_max"] in (0, 8192, 16384)
    after = ctx.run(gid, tid, 0, 8)[:2]
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    path = tmp_path / "tune.txt"
    ctx.tune_save(path)
    assert ctx.tune_load(path) >= 1
    ctx.unload_graph(gid)


# ------------------------------------------------------------------ serving

def wait_all(ctx, tickets, timeout=120):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for tk, n in tickets.items():
            if tk in res:
                continue
            r = ctx.poll(tk, n)
            if r is not None:
                res[tk] = r
        assert time.time() - t0 < timeout, "serving loop did not finish"
        time.sleep(0.001)
    return res


def mixed_workload():
    gA = I.rmat(12, 16, seed=41)
    gB = I.erdos_renyi(3000, 15000, 42)
    rng = np.random.default_rng(43)
    queries = []
    for i in range(24):
        t = int(rng.integers(3, 10))
        queries.append(dict(graph=int(rng.integers(0, 2)), t=t, edges=I.prufer_tree(t, 500 + i), k=t,
                            seed=int(rng.integers(0, 1 << 30)), first=int(rng.integers(0, 100)),
                            n=int(rng.integers(1, 20))))
    return gA, gB, queries


def test_serving_alone_equals_mixed_and_oracle(ctx):
    gA, gB, queries = mixed_workload()
    gids = [ctx.load_graph(gA), ctx.load_graph(gB)]
    tids = [ctx.load_template(q["t"], q["edges"]) for q in queries]
    # alone: one stream, one query at a time
    ctx.serve_start(max_inflight=1, max_batch=64)
    alone = []
    for q, tid in zip(queries, tids):
        tk = ctx.submit(gids[q["graph"]], tid, q["k"], q["seed"], q["first"], q["n"])
        alone.append(wait_all(ctx, {tk: q["n"]})[tk])
    ctx.serve_stop()
    # mixed: everything at once, four streams, small passes so queries split
    ctx.serve_start(max_inflight=4, max_batch=3)
    tickets = {}
    order = []
    for q, tid in zip(queries, tids):
        tk = ctx.submit(gids[q["graph"]], tid, q["k"], q["seed"], q["first"], q["n"])
        tickets[tk] = q["n"]
        order.append(tk)
    say("mixed submitted", len(order))
    mixed = wait_all(ctx, tickets)
    stats = ctx.serve_stats()
    ctx.serve_stop()
    assert stats["passes"] > len(queries)          # queries were split into several passes
    for q, a, tk in zip(queries, alone, order):
        m = mixed[tk]
        assert a["status"] == 0 and m["status"] == 0
        assert np.array_equal(a["counts"], m["counts"]) and np.array_equal(a["overflow"], m["overflow"])
        assert m["submit_s"] <= m["start_s"] <= m["done_s"]
    for q, tid, a in list(zip(queries, tids, alone))[:6]:
        g = (gA, gB)[q["graph"]]
        oc, of = oracle_for(ctx, g, gids[q["graph"]], tid, q["t"], q["k"], q["seed"], q["first"], q["n"])
        assert np.array_equal(a["counts"], oc) and np.array_equal(a["overflow"], of)
    for gid in gids:
        ctx.unload_graph(gid)


def test_serving_memory_budget_and_errors(ctx):
    g = I.rmat(13, 16, seed=44)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(10, I.prufer_tree(10, 44))
    ctx.set_colors(10, 9)
    info1 = ctx.plan_info(gid, tid, 1)
    ref = ctx.run(gid, tid, 0, 12)[:2]
    # a budget that holds about two colourings' tables at a time
    budget = int(info1.arena_bytes * 2.5) + (1 << 20)
    ctx.serve_start(mem_budget_bytes=budget, max_inflight=3, max_batch=64)
    tk = ctx.submit(gid, tid, 10, 9, 0, 12)
    r = wait_all(ctx, {tk: 12})[tk]
    stats = ctx.serve_stats()
    assert r["status"] == 0
    assert np.array_equal(r["counts"], ref[0]) and np.array_equal(r["overflow"], ref[1])
    assert stats["passes"] >= 5 and stats["peak_mem_bytes"] <= budget + (8 << 20)
    with pytest.raises(sc.ScError) as e:
        ctx.submit(gid + 99, tid, 10, 9, 0, 1)
    assert e.value.code == sc.SC_ENOTFOUND
    ctx.serve_stop()
    # a budget below one colouring: the query fails with SC_ENOMEM
    ctx.serve_start(mem_budget_bytes=1 << 20, max_inflight=2, max_batch=8)
    tk = ctx.submit(gid, tid, 10, 9, 0, 2)
    r = wait_all(ctx, {tk: 2})[tk]
    assert r["status"] == sc.SC_ENOMEM
    ctx.serve_stop()
    ctx.unload_graph(gid)
