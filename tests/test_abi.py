"""CPU-side checks of libsc: it loads, exports every symbol include/sc.h
declares, and its host logic (planner, Eq. 1 indexing, colouring rule,
automorphisms) agrees with independent computations.  No GPU needed."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*\b(sc_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    sc.lib()                                  # loads PyTorch's HIP runtime first
    L = ctypes.CDLL(sc.lib_path)
    names = declared_functions()
    assert "sc_run" in names and "sc_create" in names
    for name in names:
        assert hasattr(L, name), name


def test_version_string():
    assert "libsc" in sc.sc_version()


def test_create_requires_the_allocator_hook():
    """The allocator hook is the library's only source of device memory:
    sc_create rejects NULL hooks before it looks for a device."""
    L = sc.lib()
    h = ctypes.c_void_p()
    assert L.sc_create(0, sc.ALLOC_FN(), sc.FREE_FN(), None, 0, ctypes.byref(h)) == sc.SC_EINVAL
    assert not h.value
    keep = sc.ALLOC_FN(lambda n, s, u: None)
    assert L.sc_create(0, keep, sc.FREE_FN(), None, 0, ctypes.byref(h)) == sc.SC_EINVAL


def test_library_shares_pytorchs_hip_runtime():
    """In a fresh process, loading the library through the binding leaves one
    HIP runtime (PyTorch's) mapped."""
    import subprocess
    import sys
    code = ("from paper_1903_04395_amd import sc; sc.lib(); "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}), "
            "len({l.split()[-1] for l in m if 'libhsa-runtime64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    assert out.stdout.split() == ["1", "1"], out.stdout + out.stderr


def test_no_device_create_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sc.ScError):
        sc.Context(0)


@pytest.mark.parametrize("k", [3, 8, 12, 16])
def test_colorset_rank_matches_oracle(k):
    for m in range(0, 1 << k, max(1, (1 << k) // 4096)):
        assert sc.sc_colorset_rank(m) == O.rank(m)


@pytest.mark.parametrize("k", [3, 5, 9, 12, 16])
def test_root_step_entry_rank(k):
    """The root step (k, 1, k-1) reads, of a neighbour's row, the set of the
    k-2 renumbered colours that misses index x; its Eq. 1 rank is k-2-x (the
    oracle's rank, and the library's, of that mask)."""
    full = (1 << (k - 1)) - 1
    for x in range(k - 1):
        m = full & ~(1 << x)
        assert O.rank(m) == k - 2 - x
        assert sc.sc_colorset_rank(m) == k - 2 - x


def test_color_rule_matches_oracle():
    for seed in (0, 1, 2**63 + 5):
        for r in (0, 1, 77):
            for v in (0, 1, 12345, 2**20):
                for k in (1, 5, 12, 16):
                    assert sc.sc_color_of(seed, r, v, k) == O.color(seed, r, v, k)


def steps_of(t, root, children):
    out = []

    def rec(u):
        s = 1
        for w in children[u]:
            p = rec(w)
            out.append((s + p, s, p))
            s += p
        return s
    rec(root)
    return out


@pytest.mark.parametrize("seed", range(5))
def test_plan_steps_and_lemma1_counts(seed):
    t = 10
    edges = I.prufer_tree(t, seed)
    n, nnz, k = 1000, 8000, 10
    for root in [-1] + list(range(t)):
        info = sc.sc_plan_template(t, edges, root, k, n, nnz, 4)
        if root >= 0:
            assert info.root == root
        ch = info.children()
        # the plan is a rooted spanning tree of the template
        und = {frozenset(e) for e in edges}
        got = {frozenset((u, w)) for u in range(t) for w in ch[u]}
        assert got == und
        assert info.steps() == steps_of(t, info.root, ch)
        assert info.n_steps == t - 1
        # Lemma 1: nnz*C(k,p) neighbour-sum updates and n*C(k,h)*C(h,p)
        # multiply-adds per step; the benchmark counts an a = 1 step (a select)
        # as n*C(k,h)
        spmm = sum(nnz * math.comb(k, p) for h, a, p in info.steps())
        ema = sum(n * math.comb(k, h) * (math.comb(h, p) if a > 1 else 1) for h, a, p in info.steps())
        lemma1 = sum(nnz * math.comb(k, p) + n * math.comb(k, h) * math.comb(h, p)
                     for h, a, p in info.steps())
        assert info.spmm_updates == spmm and info.ema_updates == ema
        assert info.lemma1_ops == lemma1
        assert info.automorphisms == O.aut(t, edges)
        # executed updates in the rooted-colour layout (a row keeps only the
        # colour sets that hold its own colour): nnz*C(k-1,p-1) neighbour-sum
        # adds (nnz for p = 1) and n*C(k-1,h-1)*C(h-1,a-1) multiply-adds
        # (n*C(k-1,p) copies for a = 1)
        ex = sum((nnz * math.comb(k - 1, p - 1) if p > 1 else nnz)
                 + (n * math.comb(k - 1, h - 1) * math.comb(h - 1, a - 1) if a > 1 else n * math.comb(k - 1, p))
                 for h, a, p in info.steps())
        assert info.exec_updates == ex
        assert info.modes() == [0 if p == 1 else 1 for h, a, p in info.steps()]
        assert info.interleave in (1, 2, 4) and 4 % info.interleave == 0
        # the arena holds at least the largest step's live tables (output,
        # active and passive; single-vertex tables are implicit)
        W = lambda s: math.comb(k - 1, s - 1)
        need = max((W(h) + (W(a) if a > 1 else 0) + (W(p) if p > 1 else 0)) * n * 4 * 8
                   for h, a, p in info.steps())
        assert info.arena_bytes >= need


def test_interleave_follows_batch_and_lds():
    t, k = 12, 12
    edges = I.prufer_tree(t, 3)
    for batch, want in ((8, 8), (6, 2), (5, 1), (64, None)):
        info = sc.sc_plan_template(t, edges, -1, k, 10000, 80000, batch)
        assert batch % info.interleave == 0
        if want is not None:
            assert info.interleave <= want
    # k = 16: the neighbour-sum row of one colouring alone is C(15,7)*8 bytes
    info = sc.sc_plan_template(16, I.path(16), 0, 16, 1000, 4000, 4)
    assert info.interleave == 1


def test_planner_picks_lowest_cost_root():
    t, k = 10, 10
    edges = I.path(t)
    best = sc.sc_plan_template(t, edges, -1, k, 2**20, 31_000_000, 8)
    # the chosen plan's modelled bytes are no worse than rooting at vertex 0
    fixed = sc.sc_plan_template(t, edges, 0, k, 2**20, 31_000_000, 8)
    assert best.compulsory_bytes <= fixed.compulsory_bytes * 1.5


def test_plan_rejects_bad_templates():
    with pytest.raises(sc.ScError):
        sc.sc_plan_template(3, [(0, 1), (0, 1)], -1, 3, 10, 10, 1)
    with pytest.raises(sc.ScError):
        sc.sc_plan_template(4, I.path(4), -1, 3, 10, 10, 1)     # k < t
    with pytest.raises(sc.ScError):
        sc.sc_plan_template(17, [(i, i + 1) for i in range(16)], -1, 16, 10, 10, 1)


def test_binding_constants_match_the_header():
    """Every SC_* enumerator the binding defines has the header's value."""
    import re
    hdr = open(os.path.join(ROOT, "include", "sc.h")).read()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(SC_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr)}
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(SC_[A-Z0-9_]+)\s+(\d+)", hdr)}
    vals.update(defs)
    checked = 0
    for name in dir(sc):
        if name.startswith("SC_") and isinstance(getattr(sc, name), int) and name in vals:
            assert getattr(sc, name) == vals[name], name
            checked += 1
    assert checked >= 15
    for opt in sc.OPTION_DEFAULTS:
        assert opt in vals.values()


def test_bench_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """bench.py reports the committed HBM traffic only for the kernel sources
    it was measured on."""
    import json
    import bench
    h = bench.source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps({"source_hash": h, "hbm_bytes_per_step": 123.0}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    assert bench.traffic_per_step() == 123.0
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.traffic_per_step() is None


def test_bench_step_table_groups_launches_by_template_and_step():
    """bench.py's per-step table: a trace of two passes of one template and
    one of another is split into passes at the colour kernel, each pass
    assigned its template in call order, and times summed per step."""
    import bench
    def pass_(steps, ms):
        out = [{"family": "zero", "step": -1, "h": 0, "a": 0, "p": 0, "colorings": 8, "ms": 0.01,
                "alg_bytes": 0.0, "layout_bytes": 0.0, "updates": 0.0},
               {"family": "color", "step": -1, "h": 0, "a": 0, "p": 0, "colorings": 8, "ms": 0.02,
                "alg_bytes": 0.0, "layout_bytes": 0.0, "updates": 0.0}]
        for i, (h, a, p) in enumerate(steps):
            if p > 1:
                out.append({"family": "split", "step": i, "h": h, "a": a, "p": p, "colorings": 8, "ms": ms / 2,
                            "alg_bytes": 0.0, "layout_bytes": 1e9, "updates": 0.0})
            out.append({"family": "row_gather" if p > 1 else "row_hist", "step": i, "h": h, "a": a, "p": p,
                        "colorings": 8, "ms": ms, "alg_bytes": 8e9, "layout_bytes": 2e9, "updates": 1e9})
        return out
    t1 = [(2, 1, 1), (3, 1, 2)]
    t2 = [(2, 1, 1), (3, 2, 1)]
    trace = pass_(t1, 10.0) + pass_(t1, 10.0) + pass_(t2, 4.0)
    tab = bench.step_table(trace, ["a", "a", "b"], rows=10**7, valu={0: 1e12, 1: 2e12, 2: 3e12})
    got = {(e["template"], e["step"]): e for e in tab}
    assert set(got) == {("a", 0), ("a", 1), ("b", 0), ("b", 1)}
    # 16 colourings per step of the benchmark: the two 8-colouring passes of
    # template a make one step, the one pass of b half a step
    assert got[("a", 1)]["ms"] == pytest.approx(30.0)
    assert got[("a", 1)]["alg_GB"] == pytest.approx(16.0)
    assert got[("b", 0)]["ms"] == pytest.approx(8.0)
    assert got[("b", 1)]["G_mul_adds"] == pytest.approx(10**7 * math.comb(11, 2) * 2 * 16 / 1e9, abs=0.01)
    assert got[("b", 1)]["valu_frac"] == pytest.approx(17.6e9 / 3e12 / 8e-3, abs=2e-3)
    assert got[("a", 0)]["valu_frac"] is None and got[("b", 1)]["valu_frac"] > 0
