"""Pins of the oracle's drawing-quality metrics (Section 5.2): crossings,
edge length standard deviation, Gabriel graph and the Jaccard similarity.

Crossings: the complete graph on points in convex position has one crossing
per four vertices, C(n, 4), and an edge separating j - 1 from n - j - 1
vertices is crossed (j - 1)(n - j - 1) times; planar drawings have none;
touching and collinear cases are not crossings.  Gabriel graph: of integer
grid points it is the 4-neighbour grid (diagonals have the other two corners
on their circle); of random points it equals scipy's Delaunay edges kept by
the empty-disc test (Gabriel edges are Delaunay edges).  Jaccard: a hand
computation on collinear points.
"""
import math
from itertools import combinations

import numpy as np
import pytest
from scipy.spatial import Delaunay

import oracle
from paper_1606_02162_amd import inputs


def _polygon(n, r=100.0, phase=0.3):
    th = phase + 2 * math.pi * np.arange(n) / n
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


@pytest.mark.parametrize("n", [4, 5, 7, 10, 13])
def test_complete_graph_convex_position(n):
    g = inputs.complete_graph(n)
    pos = _polygon(n)
    total, per = oracle.crossings(g.n, g.row_ptr, g.col_idx, pos, per_edge=True)
    assert total == math.comb(n, 4)
    for e, (u, v) in enumerate(oracle.edge_list(g.row_ptr, g.col_idx)):
        j = int(v - u)
        assert per[e] == (j - 1) * (n - j - 1), (u, v)
    assert per.sum() == 2 * total


def test_planar_drawings_have_no_crossings():
    g = inputs.grid_graph(9, 11)
    pos = np.stack([np.arange(g.n) % 11, np.arange(g.n) // 11], axis=1).astype(float)
    assert oracle.crossings(g.n, g.row_ptr, g.col_idx, pos) == 0
    s = inputs.star_graph(20)
    assert oracle.crossings(s.n, s.row_ptr, s.col_idx, np.vstack([[0, 0], _polygon(20)])) == 0


def test_crossing_special_cases():
    # X: 0-1 and 2-3 cross once
    g = inputs.to_csr(4, [0, 2], [1, 3])
    x = np.array([[0, 0], [2, 2], [0, 2], [2, 0]], dtype=float)
    assert oracle.crossings(4, g.row_ptr, g.col_idx, x) == 1
    # T: the end of 2-3 touches 0-1 -> not a crossing
    x = np.array([[0, 0], [2, 0], [1, 0], [1, 2]], dtype=float)
    assert oracle.crossings(4, g.row_ptr, g.col_idx, x) == 0
    # collinear overlap -> not a crossing
    x = np.array([[0, 0], [2, 0], [1, 0], [3, 0]], dtype=float)
    assert oracle.crossings(4, g.row_ptr, g.col_idx, x) == 0
    # edges sharing an end never cross
    h = inputs.to_csr(3, [0, 0], [1, 2])
    assert oracle.crossings(3, h.row_ptr, h.col_idx, np.array([[0, 0], [1, 1], [1, -1.0]])) == 0


def test_sampled_edge_crossings_match_full():
    g = inputs.erdos_renyi(200, 500, seed=3)
    pos = inputs.uniform_positions(g.n, seed=2, width=100.0, height=100.0)
    total, per = oracle.crossings(g.n, g.row_ptr, g.col_idx, pos, per_edge=True)
    sel = np.array([0, 7, 123, per.size - 1])
    assert np.array_equal(oracle.edge_crossings(g.n, g.row_ptr, g.col_idx, pos, sel), per[sel])
    assert total > 0


def test_edge_lengths_closed_forms():
    g = inputs.path_graph(3)
    mu, sd = oracle.edge_lengths(3, g.row_ptr, g.col_idx, np.array([[0, 0], [1, 0], [1, 3.0]]))
    assert mu == 2.0 and sd == 1.0
    c = inputs.cycle_graph(16)
    mu, sd = oracle.edge_lengths(16, c.row_ptr, c.col_idx, _polygon(16, r=50.0))
    assert mu == pytest.approx(2 * 50.0 * math.sin(math.pi / 16), rel=1e-6)
    assert sd < 1e-5


def test_gabriel_of_grid_points_is_the_grid():
    rows, cols = 6, 7
    g = inputs.grid_graph(rows, cols)
    pos = np.stack([np.arange(g.n) % cols, np.arange(g.n) // cols], axis=1).astype(float)
    ptr, idx = oracle.gabriel(pos)
    assert np.array_equal(ptr, g.row_ptr) and np.array_equal(idx, g.col_idx)
    assert oracle.similarity(g.n, g.row_ptr, g.col_idx, pos) == 1.0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gabriel_random_points_against_delaunay(seed):
    x = oracle.single(np.random.default_rng(seed).uniform(0, 1000, (300, 2)))
    tri = Delaunay(x)
    cand = set()
    for s in tri.simplices:
        for a, b in combinations(sorted(int(i) for i in s), 2):
            cand.add((a, b))
    expect = set()
    for a, b in cand:
        d = ((x - x[a]) * (x - x[b])).sum(1)
        d[[a, b]] = 1.0
        if (d > 0).all():
            expect.add((a, b))
    ptr, idx = oracle.gabriel(x)
    got = {(u, int(v)) for u in range(x.shape[0]) for v in idx[ptr[u]:ptr[u + 1]] if v > u}
    assert got == expect
    assert len(got) <= 3 * x.shape[0] - 6


def test_jaccard_hand_computed():
    """Points on a line: the Gabriel graph is the path 0-1-2-3; the graph is
    the star at 0: J = 1/3, 1/2, 0, 0."""
    g = inputs.star_graph(3)
    pos = np.array([[0, 0], [1, 0], [2, 0], [3, 0]], dtype=float)
    mean, per = oracle.similarity(4, g.row_ptr, g.col_idx, pos, per_vertex=True)
    np.testing.assert_allclose(per, [1 / 3, 1 / 2, 0, 0])
    assert mean == pytest.approx(5 / 24)
