"""The (eps, delta) estimator's host side: the median-of-means bound of
sc_colorings_for against its defining inequalities and the growth Lemma 3
states, and the variance bound it rests on, Var X / (E X)^2 <= 1/P - 1, against
every colouring of small graphs (oracle counts) -- with equality where all
copies share one vertex set."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1903_04395_amd import inputs as I
from paper_1903_04395_amd import sc


def relvar_bound(k, t):
    """1/P - 1 with P = k!/((k-t)! k^t), exactly."""
    P = Fraction(math.factorial(k), math.factorial(k - t) * k**t)
    return 1 / P - 1


@pytest.mark.parametrize("k,t", [(3, 3), (5, 5), (5, 3), (10, 10), (12, 7), (16, 16)])
@pytest.mark.parametrize("eps,delta", [(0.5, 0.1), (0.1, 0.05), (0.02, 1e-6), (1.0, 0.5)])
def test_bound_meets_chebyshev_and_hoeffding_minimally(k, t, eps, delta):
    m, g = sc.colorings_for(k, t, eps, delta)
    rv = float(relvar_bound(k, t))
    assert m % 2 == 1 and m >= 1
    assert math.exp(-m / 8) <= delta * (1 + 1e-12)                  # median fails w.p. <= delta
    if m >= 3:
        assert math.exp(-(m - 2) / 8) > delta                        # no smaller odd m does
    assert rv / (g * eps**2) <= 0.25 * (1 + 1e-12)                   # a group mean fails w.p. <= 1/4
    if g > 1:
        assert rv / ((g - 1) * eps**2) > 0.25 * (1 - 1e-12)          # g is the least such


def test_bound_grows_like_e_to_the_k():
    """Lemma 3: O(e^k log(1/delta) / eps^2) colourings; for k = t the ratio
    of consecutive k tends to (1 + 1/k)^k -> e."""
    R = {k: np.prod(sc.colorings_for(k, k, 0.1, 0.01)) for k in range(3, 17)}
    for k in range(8, 16):
        assert 2.4 < R[k + 1] / R[k] < math.e * 1.001
    m1, g1 = sc.colorings_for(8, 8, 0.1, 0.01)
    m2, g2 = sc.colorings_for(8, 8, 0.05, 0.0001)
    assert abs(g2 / g1 - 4) < 0.01 and abs(m2 / m1 - 2) < 0.1       # 1/eps^2 and log(1/delta)


@pytest.mark.parametrize("bad", [(3, 4, 0.1, 0.1), (3, 3, 0.0, 0.1), (3, 3, 0.1, 1.0), (3, 3, 0.1, 0.0),
                                 (17, 3, 0.1, 0.1), (3, 3, -1.0, 0.5)])
def test_bound_rejects_bad_arguments(bad):
    with pytest.raises(sc.ScError):
        sc.colorings_for(*bad)


def all_colourings_moments(g, t, edges, k):
    plan = O.root_plan(t, edges, 0)
    xs = []
    for col in itertools.product(range(k), repeat=g.n):
        X, f = O.count_colored(g, t, plan, k, np.array(col, np.uint8))
        assert f == 0
        xs.append(int(X))
    N = len(xs)
    mean = Fraction(sum(xs), N)
    var = Fraction(sum(x * x for x in xs), N) - mean * mean
    return mean, var


def brute_maps(g, t, edges):
    """Injective maps of the tree into the graph sending edges to edges."""
    adj = [set(int(u) for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    n = 0
    for img in itertools.permutations(range(g.n), t):
        n += all(img[b] in adj[img[a]] for a, b in edges)
    return n


@pytest.mark.parametrize("case", ["k3_path3", "k4_minus_edge_path3_k4", "c5_path4", "star_graph_star3"])
def test_variance_bound_over_every_colouring(case):
    if case == "k3_path3":                                 # every map on one vertex set: equality
        g, t, edges, k = I.csr_from_edges(3, np.array([0, 0, 1]), np.array([1, 2, 2])), 3, I.path(3), 3
    elif case == "k4_minus_edge_path3_k4":
        g, t, edges, k = I.csr_from_edges(4, np.array([0, 0, 0, 1, 1]), np.array([1, 2, 3, 2, 3])), 3, I.path(3), 4
    elif case == "c5_path4":
        g, t, edges, k = I.csr_from_edges(5, np.arange(5), (np.arange(5) + 1) % 5), 4, I.path(4), 4
    else:
        g, t, edges, k = I.csr_from_edges(6, np.array([0, 0, 0, 0, 1]), np.array([1, 2, 3, 4, 5])), 3, I.star(3), 3
    mean, var = all_colourings_moments(g, t, edges, k)
    P = Fraction(math.factorial(k), math.factorial(k - t) * k**t)
    M = brute_maps(g, t, edges)
    assert mean == M * P                                   # X / P is unbiased for the maps
    bound = relvar_bound(k, t)
    assert var / (mean * mean) <= bound
    if case == "k3_path3":
        assert var / (mean * mean) == bound
    else:
        assert var / (mean * mean) < bound
