"""Host side of the command line: edge-list parsing, graph and template
construction and argument checks (no GPU)."""
import numpy as np
import pytest

from paper_1903_04395_amd import cli


def write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_read_pairs_skips_comments_and_blank_lines(tmp_path):
    p = write(tmp_path, "g.txt", "# header\n% other\n0 1\n\n1 2 7\n  2 0  \n")
    assert cli.read_pairs(p).tolist() == [[0, 1], [1, 2], [2, 0]]


@pytest.mark.parametrize("text", ["0\n", "0 -1\n", "a b\n"])
def test_read_pairs_rejects_bad_lines(tmp_path, text):
    with pytest.raises(ValueError):
        cli.read_pairs(write(tmp_path, "bad.txt", text))


def test_graph_is_simple_and_symmetric():
    g = cli.graph_from_pairs(np.array([[0, 1], [1, 0], [1, 1], [2, 3], [0, 1]]))
    assert g.n == 4 and g.nnz == 4
    assert g.col_idx[g.row_ptr[0]:g.row_ptr[1]].tolist() == [1]
    assert g.col_idx[g.row_ptr[3]:g.row_ptr[4]].tolist() == [2]


def test_template_must_be_a_tree():
    t, e = cli.template_from_pairs(np.array([[0, 1], [1, 2], [1, 3]]))
    assert t == 4 and e.dtype == np.int32
    with pytest.raises(ValueError):
        cli.template_from_pairs(np.array([[0, 1], [1, 2], [2, 0]]))        # cycle, 3 edges on 3 vertices
    with pytest.raises(ValueError):
        cli.template_from_pairs(np.array([[0, 1], [0, 1], [2, 3]]))        # repeated edge, disconnected
    with pytest.raises(ValueError):
        cli.template_from_pairs(np.array([[0, 1], [2, 3]]))                # too few edges


def test_arguments_need_colourings_or_eps():
    with pytest.raises(SystemExit):
        cli.parse(["--graph", "g", "--template", "t"])
    with pytest.raises(SystemExit):
        cli.parse(["--graph", "g", "--template", "t", "--colorings", "4", "--eps", "0.1"])
    a = cli.parse(["--graph", "g", "--template", "t", "--eps", "0.1", "--bound"])
    assert a.bound and a.colorings == 0
