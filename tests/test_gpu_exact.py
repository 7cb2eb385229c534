"""GPU parity of the exact wide counts.  The residue passes (the counting DP
with every entry taken mod p) against the oracle's modular DP, bit-exact; the
CRT-combined counts of sc_run_exact against the oracle's exact counts (Python
integers); the homomorphism bound against closed forms.  Calls go through the
C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc

pytestmark = pytest.mark.gpu

# a supported modulus that is not prime: residues need no primality
COMPOSITE = 2**62 - 1


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = sc.Context(0)
    yield c
    c.close()


def hubby_graph(seed, n=1500, m=4000, hubs=3, hub_deg=900):
    """Sparse random graph plus a few high-degree hubs, so counts pass 2^64."""
    rng = np.random.default_rng(seed)
    e = I.erdos_renyi(n, m, seed).edges()
    src, dst = [e[:, 0]], [e[:, 1]]
    for h in range(hubs):
        nb = rng.choice(np.arange(hubs, n), size=hub_deg, replace=False)
        src.append(np.full(hub_deg, h))
        dst.append(nb)
    return I.csr_from_edges(n, np.concatenate(src), np.concatenate(dst))


def setup(ctx, g, t, edges, k, seed, R, root=-1):
    gid = ctx.load_graph(g)
    tid = ctx.load_template(t, edges, root)
    ctx.set_colors(k, seed)
    info = ctx.plan_info(gid, tid, R)
    return gid, tid, info


RESIDUE_CASES = [
    # (name, graph, t, edges, k, seed, first, R, options)
    ("er_path5", lambda: I.erdos_renyi(2000, 10000, 1), 5, I.path(5), 5, 2024, 0, 8, {}),
    ("rmat12_tree10", lambda: I.rmat(12, 16, seed=2), 10, I.prufer_tree(10, 0), 10, 5, 3, 8,
     {sc.SC_OPT_SEGMENT: 128}),
    ("chunglu_tree12", lambda: I.chung_lu(3000, 20, 2.1, seed=3), 12, I.prufer_tree(12, 3), 12, 7, 0, 4, {}),
    ("hubby_star9", lambda: hubby_graph(4), 9, I.star(9), 9, 11, 1, 6, {sc.SC_OPT_SEGMENT: 256}),
    ("hubby_tree11_bi2", lambda: hubby_graph(6), 11, I.prufer_tree(11, 6), 12, 13, 0, 6,
     {sc.SC_OPT_INTERLEAVE: 2}),
    # enough rows that light steps build one row per wavefront
    ("chunglu40k_tree7_rows_per_wavefront", lambda: I.chung_lu(40000, 10, 2.2, seed=8), 7, I.prufer_tree(7, 8),
     7, 17, 0, 8, {}),
]


@pytest.mark.parametrize("case", RESIDUE_CASES, ids=[c[0] for c in RESIDUE_CASES])
def test_residues_match_the_oracle(ctx, case):
    name, mk, t, edges, k, seed, first, R, opts = case
    g = mk()
    for o, v in opts.items():
        ctx.set_option(o, v)
    try:
        gid, tid, info = setup(ctx, g, t, edges, k, seed, R)
        plan = (info.root, info.children())
        for p in O.PRIMES + (COMPOSITE,):
            say(f"{name}: n={g.n} nnz={g.nnz} t={t} k={k} R={R} batch={info.batch} p={p}")
            got = ctx.run_mod(gid, tid, first, R, p)
            want = O.count_mod(g, t, plan, k, seed, first, R, p)
            assert np.array_equal(got, want), (p, got, want)
        ctx.unload_graph(gid)
    finally:
        for o in opts:
            ctx.set_option(o, sc.OPTION_DEFAULTS[o])


# a 12-vertex spider: nine legs of length 1 and one of length 2
SPIDER = np.array([(0, i) for i in range(1, 10)] + [(0, 10), (10, 11)], np.int32)


@pytest.mark.parametrize("t,edges,root", [(12, I.star(12), 0), (12, I.star(12), 1),
                                          (12, SPIDER, -1), (12, SPIDER, 11)])
def test_exact_counts_past_2_64(ctx, t, edges, root):
    """Hub vertices push counts past 2^64; sc_run_exact recovers them exactly."""
    g = hubby_graph(9)
    k, seed, first, R = 12, 21, 2, 5
    gid, tid, info = setup(ctx, g, t, edges, k, seed, R, root)
    say(f"exact: n={g.n} nnz={g.nnz} t={t} root={info.root} R={R} batch={info.batch}")
    counts, exact, hom, maps, copies = ctx.run_exact(gid, tid, first, R)
    want = O.count_exact(g, t, (info.root, info.children()), k, seed, first, R)
    assert counts == want
    assert exact.all()
    assert max(want) >= 2**64                      # the case the residues are for
    assert hom >= max(want)
    # the uint64 pass agrees mod 2^64 and flags exactly the wide counts
    c64, ovf, _, _ = ctx.run(gid, tid, first, R)
    assert [int(x) for x in c64] == [x % 2**64 for x in want]
    assert [bool(f) for f in ovf] == [x >= 2**64 for x in want]
    P = O.colorful_probability(k, t)
    assert maps == pytest.approx(sum(want) / R / P, rel=1e-12)
    assert copies == pytest.approx(maps / O.aut(t, edges), rel=1e-12)
    ctx.unload_graph(gid)


def test_exact_without_overflow_is_the_uint64_count(ctx):
    g = I.erdos_renyi(3000, 12000, 4)
    t, k, seed, R = 7, 7, 3, 12
    gid, tid, info = setup(ctx, g, t, I.prufer_tree(7, 4), k, seed, R)
    c64, ovf, maps64, _ = ctx.run(gid, tid, 0, R)
    assert not ovf.any()
    counts, exact, hom, maps, _ = ctx.run_exact(gid, tid, 0, R)
    assert counts == [int(x) for x in c64] and exact.all()
    assert maps == pytest.approx(maps64, rel=1e-12)
    assert hom >= max(counts)
    ctx.unload_graph(gid)


def walks(g, t):
    """1^T A^(t-1) 1 in exact integers: homomorphisms of the t-vertex path."""
    x = [1] * g.n
    rp, ci = g.row_ptr, g.col_idx
    for _ in range(t - 1):
        x = [sum(x[int(u)] for u in ci[rp[v]:rp[v + 1]]) for v in range(g.n)]
    return sum(x)


@pytest.mark.parametrize("root", [0, 3])
def test_hom_count_closed_forms(ctx, root):
    """Stars: sum over v of deg(v)^(t-1); paths: 1^T A^(t-1) 1."""
    g = hubby_graph(2, n=600, m=1500, hubs=2, hub_deg=400)
    deg = [int(d) for d in g.degrees()]
    gid = ctx.load_graph(g)
    ctx.set_colors(12, 1)
    for t in (2, 5, 12):
        tid = ctx.load_template(t, I.star(t), min(root, t - 1))
        want = sum(d ** (t - 1) for d in deg)
        assert ctx.hom_count(gid, tid) == pytest.approx(want, rel=1e-12)
        tid = ctx.load_template(t, I.path(t), min(root, t - 1))
        assert ctx.hom_count(gid, tid) == pytest.approx(walks(g, t), rel=1e-12)
    ctx.unload_graph(gid)


def test_run_mod_rejects_unsupported_moduli(ctx):
    g = I.erdos_renyi(100, 300, 1)
    gid = ctx.load_graph(g)
    tid = ctx.load_template(3, I.path(3), -1)
    ctx.set_colors(3, 1)
    for p in (2**62, 2**61 - 2, 1000003, 2**64 - 59, 0):
        with pytest.raises(sc.ScError):
            ctx.run_mod(gid, tid, 0, 4, p)
    assert np.array_equal(ctx.run_mod(gid, tid, 0, 4, O.PRIMES[0]),
                          O.count_mod(g, 3, O.root_plan(3, I.path(3), 0), 3, 1, 0, 4, O.PRIMES[0]))
    ctx.unload_graph(gid)


def test_exact_counts_needing_three_primes(ctx):
    """A 6100-neighbour hub and the 16-star: the homomorphism bound (about
    2^188.6) exceeds what 2^64 and two primes certify, so all three residue
    passes run; the count (about 2^169) against the oracle's."""
    rng = np.random.default_rng(12)
    n, hub = 6200, 6100
    e = I.erdos_renyi(n, 9000, 12).edges()
    nb = rng.choice(np.arange(1, n), size=hub, replace=False)
    g = I.csr_from_edges(n, np.concatenate([e[:, 0], np.zeros(hub, np.int64)]), np.concatenate([e[:, 1], nb]))
    t = k = 16
    gid, tid, info = setup(ctx, g, t, I.star(t), k, 5, 1, root=0)
    say(f"three primes: n={g.n} nnz={g.nnz} max degree {hub}")
    counts, exact, hom, _, _ = ctx.run_exact(gid, tid, 0, 1)
    assert hom > 2.0**185
    want = O.count_exact(g, t, (info.root, info.children()), k, 5, 0, 1)
    assert counts == want and exact.all() and want[0] >= 2**124
    ctx.unload_graph(gid)


def test_degenerate_templates_and_graphs(ctx):
    """t = 1 (every vertex is a map), a graph without edges, k > t: exact counts,
    residues, the bound, the estimate and the ablation baselines agree with the
    closed forms."""
    g = I.erdos_renyi(300, 900, 2)
    empty = I.csr_from_edges(50, np.zeros(0, np.int64), np.zeros(0, np.int64))
    gid, gid0 = ctx.load_graph(g), ctx.load_graph(empty)
    t1 = ctx.load_template(1, np.zeros((0, 2), np.int32))
    t3 = ctx.load_template(3, I.path(3))
    ctx.set_colors(4, 9)
    counts, exact, hom, maps, _ = ctx.run_exact(gid, t1, 0, 3)
    assert counts == [g.n] * 3 and exact.all() and hom == g.n and maps == pytest.approx(g.n)
    assert list(ctx.run_mod(gid, t1, 0, 2, O.PRIMES[0])) == [g.n] * 2
    assert ctx.run_ablation(gid, t1, sc.SC_ABL_FASCIA, 0, 2)[0].tolist() == [g.n] * 2
    est = ctx.estimate(gid, t1, 0.1, 0.1, sc.SC_EST_SAMPLE, max_colorings=200)
    assert est.est_maps == pytest.approx(g.n) and est.exact == 1
    counts, exact, hom, _, _ = ctx.run_exact(gid0, t3, 0, 2)
    assert counts == [0, 0] and exact.all() and hom == 0
    assert ctx.run_ablation(gid0, t3, sc.SC_ABL_PFASCIA, 0, 2)[0].tolist() == [0, 0]
    # k > t: the estimate divides by k!/((k-t)! k^t)
    est = ctx.estimate(gid, t3, 0.3, 0.2, sc.SC_EST_BOUND)
    counts, _ = O.count(g, 3, O.root_plan(3, I.path(3), 0), 4, 9, 0, est.colorings)
    P = 4 * 3 * 2 / 4**3
    y = sorted(np.mean((counts.astype(float) / P).reshape(est.groups, -1)[:, :est.per_group], axis=1))
    assert est.est_maps == pytest.approx(y[est.groups // 2], rel=1e-12)
    ctx.unload_graph(gid)
    ctx.unload_graph(gid0)


@pytest.mark.parametrize("mode", [1, 2])
def test_exact_counts_replayed_from_captured_graphs(ctx, mode):
    """With SC_OPT_GRAPH the uint64 and residue passes replay captured hipGraphs
    (mode 1: one per pass shape and modulus; mode 2: one per call, its residue
    passes for every modulus in one graph); every replay, with eager work in
    between, matches the eager result."""
    g = hubby_graph(9)
    gid, tid, info = setup(ctx, g, 12, SPIDER, 12, 21, 4)
    eager = [ctx.run_exact(gid, tid, first, 4)[0] for first in (0, 4, 8)]
    ctx.set_option(sc.SC_OPT_GRAPH, mode)
    try:
        for rep in range(2):
            for i, first in enumerate((0, 4, 8)):
                got = ctx.run_exact(gid, tid, first, 4)[0]
                assert got == eager[i], (rep, first)
                ctx.set_option(sc.SC_OPT_GRAPH, 0)           # eager work between replays
                ctx.run(gid, tid, 100, 2)
                ctx.set_option(sc.SC_OPT_GRAPH, mode)
    finally:
        ctx.set_option(sc.SC_OPT_GRAPH, sc.OPTION_DEFAULTS[sc.SC_OPT_GRAPH])
    assert max(eager[0]) >= 2**64
    ctx.unload_graph(gid)


def star_closed_form(g, col, k):
    """Colourful maps of the k-vertex star (k colours) into g for one colouring:
    (k-1)! * the sum over centres v of the product, over the k-1 colours other
    than col(v), of the number of v's neighbours with that colour (exact)."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cnt = np.bincount(src * k + col[g.col_idx].astype(np.int64), minlength=g.n * k).reshape(g.n, k)
    cnt[np.arange(g.n), col] = 1
    rows = cnt[cnt.min(axis=1) > 0]
    return math.factorial(k - 1) * sum(math.prod(r) for r in rows.tolist())


# (name, n, hub degree, limbs the homomorphism bound asks for, interleave option, colourings)
WIDE_STAR_CASES = [
    ("two_limbs", 1500, 900, 2, 0, 5),
    ("three_limbs", 6000, 4000, 3, 0, 9),
    ("three_limbs_bi2", 6000, 4000, 3, 2, 4),
    ("four_limbs", 200000, 190000, 4, 0, 3),
]


@pytest.mark.parametrize("case", WIDE_STAR_CASES, ids=[c[0] for c in WIDE_STAR_CASES])
def test_exact_star_multi_limb_against_closed_form(ctx, case):
    """The 12-star rooted at its centre takes one pass whose entries carry as
    many 64-bit limbs as the homomorphism bound asks for: its counts against
    the star closed form, and (where three primes certify them) against the
    residue passes with chains switched off."""
    name, n, hub_deg, limbs, bi, R = case
    k, t, seed, first = 12, 12, 31, 1
    g = hubby_graph(17, n=n, m=2 * n, hubs=2, hub_deg=hub_deg)
    if bi:
        ctx.set_option(sc.SC_OPT_INTERLEAVE, bi)
    try:
        gid, tid, info = setup(ctx, g, t, I.star(t), k, seed, R, 0)
        say(f"wide star {name}: n={g.n} nnz={g.nnz} R={R} batch={info.batch}")
        counts, exact, hom, _, _ = ctx.run_exact(gid, tid, first, R)
        assert exact.all()
        want = [star_closed_form(g, O.colors(seed, first + r, g.n, k), k) for r in range(R)]
        assert counts == want
        assert 2 ** (64 * (limbs - 1)) <= hom * (1 + 2**-10) < 2 ** (64 * limbs)
        assert max(want) <= hom
        if hom * (1 + 2**-10) < 2**247:
            ctx.set_option(sc.SC_OPT_CHAIN, 0)
            try:
                c2, e2, _, _, _ = ctx.run_exact(gid, tid, first, R)
            finally:
                ctx.set_option(sc.SC_OPT_CHAIN, sc.OPTION_DEFAULTS[sc.SC_OPT_CHAIN])
            assert e2.all() and c2 == want
        ctx.unload_graph(gid)
    finally:
        if bi:
            ctx.set_option(sc.SC_OPT_INTERLEAVE, sc.OPTION_DEFAULTS[sc.SC_OPT_INTERLEAVE])


def test_exact_star_smaller_k_and_t(ctx):
    """A 9-star with k = 11 colours (k > t): the last step keeps binom(10, 8)
    entries per row, each of two limbs."""
    g = hubby_graph(23, n=3000, m=6000, hubs=3, hub_deg=2500)
    k, t, seed, R = 11, 9, 5, 6
    gid, tid, info = setup(ctx, g, t, I.star(t), k, seed, R, 0)
    say(f"wide star k>t: n={g.n} nnz={g.nnz} R={R} batch={info.batch}")
    counts, exact, hom, _, _ = ctx.run_exact(gid, tid, 0, R)
    want = O.count_exact(g, t, (info.root, info.children()), k, seed, 0, R)
    assert exact.all() and counts == want
    assert max(want) >= 2**64
    ctx.unload_graph(gid)


@pytest.mark.parametrize("max_batch,interleave", [(4, 0), (4, 1), (2, 2)])
def test_exact_star_multi_limb_several_passes(ctx, max_batch, interleave):
    """The multi-limb star pass folded into several passes (the last one
    partial) and at small interleaves: counts against the closed form."""
    k, t, seed, first, R = 12, 12, 41, 3, 9
    g = hubby_graph(19, n=6000, m=12000, hubs=2, hub_deg=4000)
    ctx.set_option(sc.SC_OPT_MAX_BATCH, max_batch)
    ctx.set_option(sc.SC_OPT_INTERLEAVE, interleave)
    try:
        gid, tid, info = setup(ctx, g, t, I.star(t), k, seed, R, 0)
        say(f"wide star passes: n={g.n} batch={info.batch} interleave={info.interleave} R={R}")
        assert info.batch <= max_batch
        counts, exact, hom, _, _ = ctx.run_exact(gid, tid, first, R)
        want = [star_closed_form(g, O.colors(seed, first + r, g.n, k), k) for r in range(R)]
        assert exact.all() and counts == want
        assert max(want) >= 2**64 and hom * (1 + 2**-10) >= 2**128      # three limbs at the root
        ctx.unload_graph(gid)
    finally:
        ctx.set_option(sc.SC_OPT_MAX_BATCH, sc.OPTION_DEFAULTS[sc.SC_OPT_MAX_BATCH])
        ctx.set_option(sc.SC_OPT_INTERLEAVE, sc.OPTION_DEFAULTS[sc.SC_OPT_INTERLEAVE])
