"""GPU tests of the measurement entry points: the vector-ALU probe and the
per-launch trace (families, steps, bytes and updates of every launch)."""
import math

import numpy as np
import pytest

from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = sc.Context(0)
    yield c
    c.close()


def test_valu_probe_rates(ctx):
    """Every product form runs and reports a plausible rate: above 1e11 and
    below the chip's 32-bit integer issue rate (256 CUs x 64 lanes x 2.4 GHz),
    since a multiply-add takes several instructions."""
    for form in (0, 1, 2):
        r = ctx.valu_probe(form)
        print(f"[case] valu form {form}: {r:.3e} mul-adds/s", flush=True)
        assert 1e11 < r < 256 * 64 * 2.4e9
    with pytest.raises(sc.ScError):
        ctx.valu_probe(3)


def test_trace_covers_every_step_once(ctx):
    """A traced run of a template with a chain and gather steps records per
    pass one zero, one colour, one reduce launch, one launch per unfused step
    and one per chain, with the plan's step sizes; the Lemma 1 updates sum to
    the plan's per-colouring counts times the colourings."""
    g = I.rmat(12, 16, seed=3)
    gid = ctx.load_graph(g)
    t, edges = 9, [(0, 1), (1, 2), (2, 3), (0, 4), (0, 5), (0, 6), (4, 7), (4, 8)]
    tid = ctx.load_template_plan(t, 0, [[1, 5, 6, 4], [2], [3], [], [7, 8], [], [], [], []])
    ctx.set_colors(9, 2)
    info = ctx.plan_info(gid, tid, 8)
    ctx.profile(True)
    ctx.run(gid, tid, 0, 8)
    ctx.profile(False)
    recs = ctx.profile_launches()
    fams = [r["family"] for r in recs]
    passes = -(-8 // info.batch)
    assert fams.count("zero") == passes and fams.count("color") == passes and fams.count("reduce") == passes
    assert fams.count("chain") == 2 * passes                  # leaves 5, 6 of 0 and leaves 7, 8 of 4
    kern = [r for r in recs if r["family"] in ("row_gather", "row_hist", "chain")]
    steps = info.steps()
    covered = []
    for r in kern[:len(kern) // passes]:
        if r["family"] == "chain":
            covered += [(h, h - 1, 1) for h in range(r["a"] + 1, r["h"] + 1)]
        else:
            covered.append((r["h"], r["a"], r["p"]))
    assert covered == steps
    total = sum(r["updates"] for r in recs)
    assert total == pytest.approx(8 * (info.spmm_updates + info.ema_updates), rel=1e-9)
    assert all(r["ms"] >= 0 for r in recs)
    ctx.unload_graph(gid)
