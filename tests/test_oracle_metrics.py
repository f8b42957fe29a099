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
from fractions import Fraction
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


# ---------------------------------------------------------------- exact signs
def _frac_orient(a, b, c):
    a, b, c = ([Fraction(float(t)) for t in p] for p in (a, b, c))
    d = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (d > 0) - (d < 0)


def _frac_in_disc(u, v, w):
    u, v, w = ([Fraction(float(t)) for t in p] for p in (u, v, w))
    return (w[0] - u[0]) * (w[0] - v[0]) + (w[1] - u[1]) * (w[1] - v[1]) <= 0


def _frac_crossings(edges, x):
    per = np.zeros(len(edges), dtype=np.int64)
    for i, (a, b) in enumerate(edges):
        for j, (c, d) in enumerate(edges):
            if i == j or len({a, b, c, d}) < 4:
                continue
            if (_frac_orient(x[a], x[b], x[c]) * _frac_orient(x[a], x[b], x[d]) < 0
                    and _frac_orient(x[c], x[d], x[a]) * _frac_orient(x[c], x[d], x[b]) < 0):
                per[i] += 1
    return per


def test_crossing_decided_exactly_near_tiny_coordinates():
    """A vertex at (1e-20, 2e-20): the orientation of (256, 256) against the
    edge to (512, 512) is (512 - 256)(d1 - d2), negative, but rounding each
    difference in double gives 0; the edges do cross properly."""
    d1, d2 = float(np.float32(1e-20)), float(np.float32(2e-20))
    x = np.array([[d1, d2], [512.0, 512.0], [256.0, 256.0], [0.0, 512.0]])
    g = inputs.to_csr(4, [0, 2], [1, 3])
    naive = (x[1, 0] - x[0, 0]) * (x[2, 1] - x[0, 1]) - (x[1, 1] - x[0, 1]) * (x[2, 0] - x[0, 0])
    assert naive == 0.0 and _frac_orient(x[0], x[1], x[2]) == -1
    assert oracle.crossings(4, g.row_ptr, g.col_idx, x) == 1
    # mirrored: the point lies on the other side, still a crossing
    x2 = x.copy()
    x2[0] = [d2, d1]
    x2[3] = [512.0, 0.0]
    assert _frac_orient(x2[0], x2[1], x2[2]) == 1
    assert oracle.crossings(4, g.row_ptr, g.col_idx, x2) == 1


def test_gabriel_disc_decided_exactly():
    """u = (1e-20, 0), v = (2, 0), w = (1, 1): (w - u).(w - v) equals the tiny
    x-coordinate of u, so w is just outside the disc on uv (rounded
    differences give 0, inside); all three pairs are Gabriel edges."""
    d = float(np.float32(1e-20))
    x = np.array([[d, 0.0], [2.0, 0.0], [1.0, 1.0]])
    assert not _frac_in_disc(x[0], x[1], x[2])
    assert (x[2, 0] - x[0, 0]) * (x[2, 0] - x[1, 0]) + (x[2, 1] - x[0, 1]) * (x[2, 1] - x[1, 1]) == 0.0
    ptr, idx = oracle.gabriel(x)
    assert list(ptr) == [0, 2, 4, 6]
    x[0, 0] = -d  # now w is inside: u and v are not adjacent
    ptr, idx = oracle.gabriel(x)
    assert list(idx[ptr[0]:ptr[1]]) == [2]


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_exact_signs_on_near_degenerate_drawings(seed):
    """Points drawn from a few coordinate values of very different
    magnitudes (many collinear and cocircular triples, coincident points):
    crossings per edge and the Gabriel graph against exact rational
    arithmetic."""
    rng = np.random.default_rng(seed)
    vals = np.float32([0.0, 1e-20, -3e-20, 1.0, 2.0, 3.0, 1e-7, 1024.0, 1024.0000001, 5e9])
    n = 11
    x = vals[rng.integers(0, vals.size, (n, 2))].astype(np.float64)
    g = inputs.erdos_renyi(n, 22, seed=seed)
    edges = [tuple(e) for e in oracle.edge_list(g.row_ptr, g.col_idx)]
    tot, per = oracle.crossings(g.n, g.row_ptr, g.col_idx, x, per_edge=True)
    expect = _frac_crossings(edges, x)
    assert np.array_equal(per, expect) and tot == expect.sum() // 2
    ptr, idx = oracle.gabriel(x)
    for u in range(n):
        want = [v for v in range(n) if v != u and not any(
            _frac_in_disc(x[u], x[v], x[w]) for w in range(n) if w not in (u, v))]
        assert list(idx[ptr[u]:ptr[u + 1]]) == want, u


def test_jaccard_of_vertices_with_empty_neighbourhoods():
    """Three coincident points: every disc on one of them holds another (on
    its boundary), so none has a Gabriel neighbour; without graph edges
    their Jaccard index is 1 (both sets empty).  A vertex with Gabriel
    neighbours but no graph edges has index 0."""
    g = inputs.to_csr(5, [3], [4])
    x = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [5.0, 0.0], [5.0, 3.0]])
    ptr, idx = oracle.gabriel(x)
    assert list(ptr) == [0, 0, 0, 0, 1, 2]
    mean, per = oracle.similarity(5, g.row_ptr, g.col_idx, x, per_vertex=True)
    assert list(per) == [1.0, 1.0, 1.0, 1.0, 1.0] and mean == 1.0
    h = inputs.to_csr(3, [0], [1])
    y = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 5.0]])
    _, per = oracle.similarity(3, h.row_ptr, h.col_idx, y, per_vertex=True)
    np.testing.assert_allclose(per, [0.5, 0.5, 0.0])
