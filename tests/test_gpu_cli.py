"""GPU: the command line end to end on edge-list files; its estimate against
the oracle's estimate from the same colourings."""
import json

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import cli
from paper_1903_04395_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_cli_counts_from_files(tmp_path, capsys):
    g = I.erdos_renyi(400, 1600, 13)
    gp = tmp_path / "g.txt"
    gp.write_text("# ER(400, 1600)\n" + "\n".join(f"{u} {v}" for u, v in g.edges()) + "\n")
    edges = I.prufer_tree(6, 2)
    tp = tmp_path / "t.txt"
    tp.write_text("\n".join(f"{u} {v}" for u, v in edges) + "\n")
    out = cli.main(["--graph", str(gp), "--template", str(tp), "--colorings", "16", "--seed", "5"])
    assert json.loads(capsys.readouterr().out.strip().splitlines()[-1]) == json.loads(json.dumps(out))
    assert out["t"] == 6 and out["k"] == 6 and out["exact"]
    g2 = cli.graph_from_pairs(cli.read_pairs(str(gp)))
    assert g2.nnz == g.nnz
    counts, flags = O.count(g2, 6, O.root_plan(6, edges, 0), 6, 5, 0, 16)
    maps, copies = O.estimate(counts, flags, 6, 6, O.aut(6, edges))
    assert out["est_maps"] == pytest.approx(maps, rel=1e-12)
    assert out["est_copies"] == pytest.approx(copies, rel=1e-12)
    e = cli.main(["--graph", str(gp), "--template", str(tp), "--eps", "0.2", "--delta", "0.2",
                  "--max-colorings", "4000"])
    assert e["exact"] and e["colorings"] <= 4000 and abs(e["est_maps"] - maps) <= 0.5 * maps
