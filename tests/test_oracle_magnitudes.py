"""Pins of the oracle's per-vertex sum of term magnitudes S_v.

S_v = sum over adjacent u of ||f^a|| = delta^p / d plus sum over u in N_v(k)
of w_u ||f^r|| = w_u d^2 / delta^q (Section 3.1 magnitudes, Section 4.5
k-neighbourhood, Section 4.6 weights).  It is the scale of the per-vertex
force gate and the numerator of the condition number kappa_v = S_v / |F_v|.
The pins are hand-derived closed forms (two vertices, a ring on a regular
polygon, a star), the triangle inequality against the force, and exact
special cases; none retypes the per-term formula.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1606_02162_amd import inputs


def _S(g, k, d, pos, mass=None, p=2, q=1):
    kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
    return oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, kp, ki, d, pos, mass=mass, p=p, q=q)


@pytest.mark.parametrize("p,q", [(2, 1), (0, 1), (1, 2), (3, 0), (4, 5)])
@pytest.mark.parametrize("delta", [0.5, 3.0, 17.0])
def test_two_vertices_closed_form(p, q, delta):
    """One edge of length delta: each end has one attraction term of
    magnitude delta^p / d and one repulsion term of magnitude d^2 / delta^q."""
    d = 6.0
    g = inputs.path_graph(2)
    pos = np.array([[2.0, -1.0], [2.0 + 0.6 * delta, -1.0 + 0.8 * delta]])
    S = _S(g, 2, d, pos, p=p, q=q)
    want = delta ** p / d + d * d / delta ** q
    np.testing.assert_allclose(S, [want, want], rtol=1e-13)


@pytest.mark.parametrize("n", [7, 12])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_ring_regular_polygon_closed_form(n, k):
    """C_n on a regular polygon of radius R (2k < n): a vertex's k-hop
    neighbours sit at ring offsets +-1..+-k, at chord 2R sin(pi j / n); its
    two edges have the side 2R sin(pi / n)."""
    d, R = 4.0, 9.0
    g = inputs.cycle_graph(n)
    th = 2 * math.pi * np.arange(n) / n + 0.2
    pos = np.stack([R * np.cos(th), R * np.sin(th)], axis=1)
    S = _S(g, k, d, pos)
    side = 2 * R * math.sin(math.pi / n)
    want = 2 * side * side / d + 2 * sum(d * d / (2 * R * math.sin(math.pi * j / n))
                                         for j in range(1, k + 1))
    np.testing.assert_allclose(S, want, rtol=1e-12)


@pytest.mark.parametrize("k", [1, 2])
def test_star_closed_form(k):
    """K_{1,m}, hub at the centre and leaves evenly on a circle of radius R:
    the hub has m terms of each kind (R^2/d and d^2/R); a leaf has the hub's
    pair of terms and, for k >= 2, one repulsion d^2 / (2R sin(pi j / m)) per
    other leaf at angular offset j."""
    m, d, R = 9, 5.0, 3.0
    g = inputs.star_graph(m)
    th = 2 * math.pi * np.arange(m) / m
    pos = np.zeros((m + 1, 2))
    pos[0] = [1.5, -2.5]
    pos[1:, 0] = pos[0, 0] + R * np.cos(th)
    pos[1:, 1] = pos[0, 1] + R * np.sin(th)
    S = _S(g, k, d, pos)
    np.testing.assert_allclose(S[0], m * (R * R / d + d * d / R), rtol=1e-13)
    leaf = R * R / d + d * d / R
    if k >= 2:
        leaf += sum(d * d / (2 * R * math.sin(math.pi * j / m)) for j in range(1, m))
    np.testing.assert_allclose(S[1:], leaf, rtol=1e-12)


def test_zero_weights_leave_attraction_only():
    """With every repulsion weight 0 only the attraction magnitudes remain: a
    star's hub then has m R^2 / d."""
    m, d, R = 6, 2.0, 7.0
    g = inputs.star_graph(m)
    th = 2 * math.pi * np.arange(m) / m
    pos = np.zeros((m + 1, 2))
    pos[1:, 0] = R * np.cos(th)
    pos[1:, 1] = R * np.sin(th)
    S = _S(g, 2, d, pos, mass=np.zeros(m + 1))
    np.testing.assert_allclose(S[0], m * R * R / d, rtol=1e-13)
    np.testing.assert_allclose(S[1:], R * R / d, rtol=1e-13)


def test_bounds_the_force_on_random_graphs():
    """|F_v| <= S_v (triangle inequality), for every vertex of random graphs
    and force models; equality fails only by rounding."""
    for seed, (p, q) in enumerate([(2, 1), (0, 1), (2, 2), (1, 3)]):
        g = inputs.erdos_renyi(400, 900, seed=seed + 10)
        pos = inputs.uniform_positions(g.n, seed, 500.0)
        kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, 2)
        F, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 30.0, pos, p=p, q=q)
        S = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, kp, ki, 30.0, pos, p=p, q=q)
        assert np.all(np.hypot(F[:, 0], F[:, 1]) <= S * (1 + 1e-12))


def test_path_on_a_line_by_hand():
    """The path 0 - 1 - 2 with k = 2 laid out on the x axis at 0, -2 and 5:
    vertex 2 has its edge to 1 (length 7) and the 2-hop neighbour 0 (at 5);
    vertex 0 has its edge to 1 (length 2) and the 2-hop neighbour 2 (at 5).
    Each magnitude is written out by hand."""
    d = 3.0
    g = inputs.path_graph(3)
    pos = np.array([[0.0, 0.0], [-2.0, 0.0], [5.0, 0.0]])
    S = _S(g, 2, d, pos)
    np.testing.assert_allclose(S[2], 49.0 / d + 9.0 / 7.0 + 9.0 / 5.0, rtol=1e-14)
    np.testing.assert_allclose(S[0], 4.0 / d + 9.0 / 2.0 + 9.0 / 5.0, rtol=1e-14)
    # vertex 1: edges to 0 (length 2) and 2 (length 7), the same two in N_1(2)
    np.testing.assert_allclose(S[1], 4.0 / d + 49.0 / d + 9.0 / 2.0 + 9.0 / 7.0, rtol=1e-14)


def test_coincident_and_isolated_contribute_nothing():
    """A coincident neighbour adds no magnitude (it exerts no force); an
    isolated vertex has S = 0."""
    g = inputs.to_csr(4, [0, 1], [1, 2])
    pos = np.array([[0.0, 0.0], [0.0, 0.0], [3.0, 4.0], [9.0, 9.0]])
    S = _S(g, 2, 10.0, pos)
    # vertex 0: neighbour 1 coincident (nothing), 2-hop neighbour 2 at distance 5
    np.testing.assert_allclose(S[0], 100.0 / 5.0, rtol=1e-14)
    assert S[3] == 0.0


def test_sampled_rows_match_full():
    g = inputs.barabasi_albert(600, 3, seed=2)
    pos = inputs.uniform_positions(g.n, 1, 800.0)
    kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, 3)
    full = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, kp, ki, 20.0, pos)
    verts = np.array([5, 0, 599, 17, 17], dtype=np.int32)
    sp, si = oracle.khop(g.n, g.row_ptr, g.col_idx, 3, verts=verts)
    sub = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, sp, si, 20.0, pos, verts=verts)
    assert np.array_equal(sub, full[verts])


def test_nonuniform_weights_are_the_neighbours():
    """The repulsion magnitude of u on v is scaled by u's weight (the repulsion
    u exerts, Section 4.6), not v's: a star's hub with k = 1 then has
    sum_i (R^2 / d + w_i d^2 / R) over its leaves i, and leaf i has
    R^2 / d + w_hub d^2 / R."""
    m, d, R = 5, 2.0, 4.0
    g = inputs.star_graph(m)
    th = 2 * math.pi * np.arange(m) / m + 0.4
    pos = np.zeros((m + 1, 2))
    pos[1:, 0] = R * np.cos(th)
    pos[1:, 1] = R * np.sin(th)
    w = np.array([3.0, 1.0, 2.0, 5.0, 0.5, 7.0])
    S = _S(g, 1, d, pos, mass=w)
    np.testing.assert_allclose(S[0], sum(R * R / d + wi * d * d / R for wi in w[1:]), rtol=1e-13)
    np.testing.assert_allclose(S[1:], R * R / d + w[0] * d * d / R, rtol=1e-13)
