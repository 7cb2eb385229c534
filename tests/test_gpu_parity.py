"""GPU parity: libsc's HIP path against the CPU oracle, colouring by colouring,
bit-exact on (count mod 2^64, overflow flag).  Calls go through the C ABI
(ctypes binding); the oracle follows the plan the library reports."""
import math

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


def run_both(ctx, g, t, edges, k, seed, first, R, root=-1, gid=None, plan=None, opts=None):
    opts = opts or {}
    for o, v in opts.items():
        ctx.set_option(o, v)
    try:
        own_graph = gid is None
        if own_graph:
            gid = ctx.load_graph(g)
        if plan is not None:
            tid = ctx.load_template_plan(t, plan[0], plan[1])
        else:
            tid = ctx.load_template(t, edges, root)
        ctx.set_colors(k, seed)
        info = ctx.plan_info(gid, tid, R)
        say(f"n={g.n} nnz={g.nnz} t={t} k={k} seed={seed} first={first} R={R} batch={info.batch} "
            f"root={info.root} steps={info.steps()} modes={info.modes()} opts={opts}")
        counts, ovf, maps, copies = ctx.run(gid, tid, first, R)
        ocounts, oflags = O.count(g, t, (info.root, info.children()), k, seed, first, R)
        assert np.array_equal(counts, ocounts), (counts, ocounts)
        assert np.array_equal(ovf, oflags), (ovf, oflags)
        if own_graph:
            ctx.unload_graph(gid)
        return counts, ovf, maps, copies, info
    finally:
        for o in opts:
            ctx.set_option(o, sc.OPTION_DEFAULTS[o])


# ------------------------------------------------------------------ configs

def test_config1_er2000_p5_endpoint(ctx):
    """ER G(2000, 10000), 5-vertex path rooted at an endpoint, k = 5."""
    g = I.erdos_renyi(2000, 10000, seed=1)
    counts, ovf, maps, copies, info = run_both(ctx, g, 5, I.path(5), 5, 2024, 0, 16, root=0)
    assert info.root == 0 and not ovf.any()
    assert all(s[1] == 1 for s in info.steps())          # all a = 1 steps
    omaps, ocopies = O.estimate(counts, ovf, 5, 5, O.aut(5, I.path(5)))
    assert maps == pytest.approx(omaps, rel=1e-12) and copies == pytest.approx(ocopies, rel=1e-12)


def test_config2_shape_rmat_k10_batch8(ctx):
    """RMAT (scale reduced to 13), 10-vertex Pruefer tree, k = 10, 8 colourings
    folded into one pass; hubs exceed the segment so split rows run too."""
    g = I.rmat(13, 16, seed=2)
    run_both(ctx, g, 10, I.prufer_tree(10, 0), 10, 5, 0, 8)
    run_both(ctx, g, 10, I.prufer_tree(10, 1), 10, 6, 8, 8, opts={sc.SC_OPT_SEGMENT: 128})


def test_config3_shape_chunglu_k12(ctx):
    """Chung-Lu power law (n reduced to 4096), 12-vertex tree and 12-star, k = 12."""
    g = I.chung_lu(4096, 30, 2.1, seed=3)
    run_both(ctx, g, 12, I.prufer_tree(12, 3), 12, 7, 0, 4)
    run_both(ctx, g, 12, I.star(12), 12, 7, 0, 4, root=0)


def test_config4_shape_rmat_k15(ctx):
    """RMAT (scale reduced to 9), 15-vertex tree, k = 15 (6435-column tables)."""
    g = I.rmat(9, 16, seed=4)
    run_both(ctx, g, 15, I.prufer_tree(15, 4), 15, 9, 0, 2)


@pytest.mark.parametrize("shape", ["path", "tree"])
def test_k16_rows_beyond_64kb_lds(ctx, shape):
    """k = 16: a neighbour-sum row of one colouring holds up to C(15,7) = 6435
    entries, so with its index tables a row kernel needs more than 64 KB of
    LDS (the largest templates the library takes)."""
    g = I.rmat(7, 8, seed=16)
    edges = I.path(16) if shape == "path" else I.prufer_tree(16, 16)
    run_both(ctx, g, 16, edges, 16, 21, 0, 2, root=0)


# ------------------------------------------------------------------ sweeps

@pytest.mark.parametrize("seed", range(6))
def test_random_sweep(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(30, 3000))
    m = int(min(n * (n - 1) // 2, n * rng.uniform(1, 12)))
    g = I.erdos_renyi(n, m, seed)
    t = int(rng.integers(2, 9))
    edges = I.prufer_tree(t, seed + 100)
    k = t + int(rng.integers(0, 2))
    R = int(rng.integers(1, 12))
    gid = ctx.load_graph(g)
    for root in range(t):
        run_both(ctx, g, t, edges, k, seed, root * 3, R, root=root, gid=gid)
    ctx.unload_graph(gid)


@pytest.mark.parametrize("B", [1, 3, 6, 8, 12])
def test_batch_sizes_agree(ctx, B):
    g = I.rmat(11, 16, seed=9)
    run_both(ctx, g, 7, I.prufer_tree(7, 9), 7, 11, 5, 9, opts={sc.SC_OPT_MAX_BATCH: B})


@pytest.mark.parametrize("seg", [65, 200, 4096])
def test_segment_sizes_agree(ctx, seg):
    g = I.rmat(12, 16, seed=10)
    run_both(ctx, g, 8, I.prufer_tree(8, 10), 8, 12, 0, 4, opts={sc.SC_OPT_SEGMENT: seg})


@pytest.mark.parametrize("inter,lds", [(1, 0), (2, 0), (4, 0), (8, 0), (8, 16384), (2, 163840)])
def test_interleave_and_lds_limits_agree(ctx, inter, lds):
    """Colourings interleaved per table plane, and active rows staged in LDS
    or read from global memory (a 16 KB limit forces the latter)."""
    g = I.rmat(11, 16, seed=12)
    run_both(ctx, g, 9, I.prufer_tree(9, 12), 9, 13, 0, 8,
             opts={sc.SC_OPT_INTERLEAVE: inter, sc.SC_OPT_LDS_MAX: lds})


@pytest.mark.parametrize("wave_rows,scale,inter", [(0, 16, 0), (40960, 16, 0), (40960, 13, 1)])
def test_row_per_workgroup_or_per_wavefront_agree(ctx, wave_rows, scale, inter):
    """Every step built with one row per workgroup (0), or with one row per
    wavefront wherever the row fits (40960 bytes).  Rows per wavefront need
    enough (plane, row) items to fill the chip: RMAT-16 with 8 interleaved
    colourings, or RMAT-13 with 8 planes of one."""
    g = I.rmat(scale, 16, seed=13)
    run_both(ctx, g, 10, I.prufer_tree(10, 13), 10, 14, 0, 8,
             opts={sc.SC_OPT_WAVE_ROW_MAX: wave_rows, sc.SC_OPT_INTERLEAVE: inter})


# ------------------------------------------------------------------ chains of single-vertex attaches

def spider(legs):
    """Centre 0 with one path (leg) of each given length."""
    edges, nxt = [], 1
    for L in legs:
        prev = 0
        for _ in range(L):
            edges.append((prev, nxt))
            prev, nxt = nxt, nxt + 1
    return nxt, edges


CHAIN_CASES = [
    # (name, t, edges, root, k, explicit plan): runs of leaf children fused into one kernel
    ("star8", 8, I.star(8), 0, 8, None),
    ("star11_k12", 11, I.star(11), 0, 12, None),
    # the leg first, then four leaves: a chain whose first active table is
    # the gather step's output (a0 = 4)
    ("spider_leg_then_leaves", *spider([3, 1, 1, 1, 1]), 0, 9, (0, [[1, 4, 5, 6, 7], [2], [3], [], [], [], [], []])),
    ("spider_leaves_then_leg", *spider([1, 1, 1, 2]), 0, 7, None),
    ("tree12_seed3", 12, I.prufer_tree(12, 3), -1, 12, None),
]


@pytest.mark.parametrize("name,t,edges,root,k,plan", CHAIN_CASES, ids=[c[0] for c in CHAIN_CASES])
@pytest.mark.parametrize("chain", [1, 0])
def test_chains_fused_or_per_step_match_oracle(ctx, name, t, edges, root, k, plan, chain):
    """Runs of single-vertex attaches as one chain kernel (intermediate tables
    in LDS) or one kernel per step: both equal the oracle, on a power-law
    graph with rows above the segment size (their colour counts come from the
    split pre-pass), with 1, 2 and 8 interleaved colourings."""
    g = I.chung_lu(3000, 20, 2.1, seed=5)
    for inter in (1, 2, 8):
        run_both(ctx, g, t, edges, k, 31, 5, 8, root=root, plan=plan,
                 opts={sc.SC_OPT_CHAIN: chain, sc.SC_OPT_INTERLEAVE: inter, sc.SC_OPT_SEGMENT: 100})


def test_chain_overflow_flags_and_residues(ctx):
    """A star whose count passes 2^64 on K_{1,d} plus a hub graph: the chain
    kernel's flags and residues equal the oracle's and the per-step path's;
    its residue passes (mod p) equal the oracle's modular DP."""
    d = 300
    g = I.csr_from_edges(d + 1, np.zeros(d, np.int64), np.arange(1, d + 1))
    c1 = run_both(ctx, g, 12, I.star(12), 12, 3, 0, 8, root=0, opts={sc.SC_OPT_CHAIN: 1})
    c0 = run_both(ctx, g, 12, I.star(12), 12, 3, 0, 8, root=0, opts={sc.SC_OPT_CHAIN: 0})
    assert c1[1].all() and np.array_equal(c1[0], c0[0])
    gid = ctx.load_graph(g)
    tid = ctx.load_template(12, I.star(12), 0)
    ctx.set_colors(12, 3)
    info = ctx.plan_info(gid, tid, 8)
    for p in O.PRIMES:
        got = ctx.run_mod(gid, tid, 0, 8, p)
        want = O.count_mod(g, 12, (info.root, info.children()), 12, 3, 0, 8, p)
        assert np.array_equal(got, want), p
    ctx.unload_graph(gid)


@pytest.mark.parametrize("tmpl,seg,inter", [("path", 0, 0), ("path", 128, 1), ("star_leaf", 128, 8),
                                            ("star_leaf", 0, 2)])
def test_root_step_kernel_matches_oracle(ctx, tmpl, seg, inter):
    """A template on all k colours whose root has one leaf child ends in the
    step (k, 1, k-1), which reads one word of each neighbour's row and sums
    rows of every degree itself: counts and flags (hub rows past the segment
    size, counts past 2^64) and residues against the oracle, and the traced
    kernel is the root-step kernel."""
    rng = np.random.default_rng(5)
    base = I.erdos_renyi(1200, 5000, 5)
    e = base.edges()
    src, dst = [e[:, 0]], [e[:, 1]]
    for h in range(4):
        nb = rng.choice(np.arange(4, 1200), size=900, replace=False)
        src.append(np.full(900, h))
        dst.append(nb)
    g = I.csr_from_edges(1200, np.concatenate(src), np.concatenate(dst))
    t = k = 9
    # rooted at an endpoint or at a leaf of the star: the last step is (9, 1, 8)
    edges, root = (I.path(t), 0) if tmpl == "path" else (I.star(t), 1)
    opts = {sc.SC_OPT_SEGMENT: seg, sc.SC_OPT_INTERLEAVE: inter}
    counts, ovf, _, _, info = run_both(ctx, g, t, edges, k, 23, 2, 8, root=root, opts=opts)
    assert tuple(info.steps()[-1]) == (k, 1, k - 1)
    if tmpl == "star_leaf":
        assert ovf.any()                        # the hubs push the star's counts past 2^64
    for o, v in opts.items():
        ctx.set_option(o, v)
    try:
        gid = ctx.load_graph(g)
        tid = ctx.load_template(t, edges, root)
        ctx.set_colors(k, 23)
        ctx.profile(True)
        ctx.run(gid, tid, 2, 8)
        ctx.profile(False)
        last = [r for r in ctx.profile_launches() if r["family"] == "row_gather" and r["h"] == k]
        assert last and all(r["kernel"].startswith("dp_root_kernel") for r in last)
        for p in O.PRIMES[:2]:
            got = ctx.run_mod(gid, tid, 2, 8, p)
            want = O.count_mod(g, t, (info.root, info.children()), k, 23, 2, 8, p)
            assert np.array_equal(got, want), p
        ctx.unload_graph(gid)
    finally:
        for o in opts:
            ctx.set_option(o, sc.OPTION_DEFAULTS[o])


# ------------------------------------------------------------------ overflow and edge cases

def test_overflow_flags_match(ctx):
    rng = np.random.default_rng(3)
    base = I.erdos_renyi(1500, 4000, 3)
    e = base.edges()
    src, dst = [e[:, 0]], [e[:, 1]]
    for h in range(8):
        nb = rng.choice(np.arange(8, 1500), size=1400, replace=False)
        src.append(np.full(1400, h))
        dst.append(nb)
    g = I.csr_from_edges(1500, np.concatenate(src), np.concatenate(dst))
    counts, ovf, maps, copies, _ = run_both(ctx, g, 11, I.prufer_tree(11, 3), 11, 17, 0, 6)
    assert ovf.any() and math.isnan(maps)


def test_overflow_boundary_star(ctx):
    t = k = 12
    for bump in (0, 5, 6, 11):
        ns = [11] * 11
        for i in range(bump):
            ns[i] += 1
        d = sum(ns)
        g = I.csr_from_edges(d + 1, np.zeros(d, np.int64), np.arange(1, d + 1))
        # colours are drawn by the library's rule; the oracle follows the same rule
        run_both(ctx, g, t, I.star(t), k, bump, 0, 3, root=0)


def test_edge_cases(ctx):
    iso = I.csr_from_edges(7, np.array([0, 1]), np.array([1, 2]))
    run_both(ctx, iso, 1, [], 1, 1, 0, 2, root=0)              # t = 1: X = n
    run_both(ctx, iso, 2, [(0, 1)], 2, 1, 0, 5)                 # single step
    run_both(ctx, iso, 3, I.path(3), 4, 2, 0, 3)                 # k > t
    lone = I.csr_from_edges(1, np.array([], np.int64), np.array([], np.int64))
    run_both(ctx, lone, 3, I.path(3), 3, 3, 0, 2)                # no edges at all
    run_both(ctx, I.erdos_renyi(100, 300, 5), 4, I.star(4), 4, 4, 0, 0)   # zero colourings


def test_invalid_inputs_rejected(ctx):
    with pytest.raises(sc.ScError) as e:
        ctx.load_graph_csr(3, np.array([0, 1, 1, 1]), np.array([1]))     # asymmetric
    assert e.value.code == sc.SC_EINVAL
    with pytest.raises(sc.ScError):
        ctx.load_graph_csr(2, np.array([0, 1, 2]), np.array([0, 1]))     # self-loops
    with pytest.raises(sc.ScError):
        ctx.load_template(3, [(0, 1), (0, 1)])                           # not a tree
    gid = ctx.load_graph(I.erdos_renyi(20, 30, 1))
    tid = ctx.load_template(4, I.path(4))
    ctx.set_colors(3, 1)
    with pytest.raises(sc.ScError):
        ctx.run(gid, tid, 0, 1)                                          # k < t
    with pytest.raises(sc.ScError) as e:
        ctx.run(gid + 999, tid, 0, 1)
    assert e.value.code == sc.SC_ENOTFOUND
    ctx.unload_graph(gid)


# ------------------------------------------------------------------ invariances at full size

def test_full_config2_batch_and_plan_invariance(ctx):
    """RMAT scale 20 (1,048,576 vertices), 10-vertex tree, k = 10, the 8
    colourings of one pass.  At this size the oracle is timed elsewhere; here
    the properties that hold at any size are checked: the batched pass equals
    eight single-colouring passes (residue and flag), and a different root
    gives the same residues."""
    g = I.rmat(20, 16, seed=0)
    t = k = 10
    edges = I.prufer_tree(t, 0)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(t, edges)
    ctx.set_colors(k, 1)
    say("full config2 batched")
    c8, f8, _, _ = ctx.run(gid, tid, 0, 8)
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 1)
    say("full config2 single")
    c1, f1, _, _ = ctx.run(gid, tid, 0, 8)
    ctx.set_option(sc.SC_OPT_MAX_BATCH, 64)
    assert np.array_equal(c8, c1) and np.array_equal(f8, f1)
    info = ctx.plan_info(gid, tid, 8)
    other = (info.root + 1) % t
    tid2 = ctx.load_template(t, edges, root=other)
    say("full config2 other root")
    c2, _, _, _ = ctx.run(gid, tid2, 0, 8)
    assert np.array_equal(c8, c2)
    ctx.unload_graph(gid)


def test_relabelling_does_not_change_results(ctx):
    """Graphs are kept relabelled by descending degree (SC_OPT_REORDER 1), in
    reverse Cuthill-McKee order (2) or as given (0); colours follow the caller's
    ids, so residues and flags agree."""
    g = I.rmat(12, 16, seed=21)
    out = []
    for reorder in (0, 1, 2):
        ctx.set_option(sc.SC_OPT_REORDER, reorder)
        gid = ctx.load_graph(g)
        out.append(run_both(ctx, g, 9, I.prufer_tree(9, 21), 9, 3, 0, 6, gid=gid)[:2])
        ctx.unload_graph(gid)
    with pytest.raises(sc.ScError):
        ctx.set_option(sc.SC_OPT_REORDER, 3)
    ctx.set_option(sc.SC_OPT_REORDER, 1)
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0]) and np.array_equal(out[0][1], o[1])
