"""Pins of the oracle's pruning, leaf-weighted repulsion and reinsertion.

Pruning removes the degree-one vertices once, right after loading, and keeps
per vertex the number removed from it (Section 4.3).  During the layout the
repulsion a vertex exerts grows with that number (Section 4.6; weight read as
1 + leaves).  Afterwards the leaves go back on a circle of radius 0.2 times
the vertex's shortest incident edge, spread uniformly and away from the
incident edges (Section 4.6).

The pins are hand-derived small cases, brute force on a dense adjacency
matrix, an exact weighted action-reaction identity, and a grid search over
the rotation of the leaf circle.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1606_02162_amd import inputs


def _dense(g):
    A = np.zeros((g.n, g.n), dtype=bool)
    for v in range(g.n):
        A[v, g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]] = True
    return A


# -------------------------------------------------------------------- pruning

def test_prune_star():
    g = inputs.star_graph(5)  # centre 0, leaves 1..5
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    assert pr.n == 1
    assert list(pr.anchor) == [-1, 0, 0, 0, 0, 0]
    assert list(pr.leaves) == [5, 0, 0, 0, 0, 0]
    assert list(pr.new_id) == [0, -1, -1, -1, -1, -1]
    assert list(pr.row_ptr) == [0, 0] and pr.col_idx.size == 0
    assert list(pr.mass()) == [6.0]


def test_prune_path():
    g = inputs.path_graph(5)  # 0-1-2-3-4: the two ends go, one pass only
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    assert list(pr.anchor) == [1, -1, -1, -1, 3]
    assert list(pr.leaves) == [0, 1, 0, 1, 0]
    assert list(pr.new_id) == [-1, 0, 1, 2, -1]
    assert pr.n == 3
    assert list(pr.row_ptr) == [0, 1, 3, 4]
    assert list(pr.col_idx) == [1, 0, 2, 1]
    assert list(pr.mass()) == [2.0, 1.0, 2.0]


def test_prune_isolated_edge_and_vertex():
    """An isolated edge keeps its smaller end; an isolated vertex stays."""
    g = inputs.to_csr(4, [1], [3])  # vertices 0 and 2 isolated
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    assert list(pr.anchor) == [-1, -1, -1, 1]
    assert list(pr.leaves) == [0, 1, 0, 0]
    assert list(pr.new_id) == [0, 1, 2, -1]
    assert pr.n == 3 and pr.col_idx.size == 0


def test_prune_empty_graph():
    g = inputs.to_csr(0, [], [])
    pr = oracle.prune(0, g.row_ptr, g.col_idx)
    assert pr.n == 0 and pr.row_ptr.tolist() == [0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prune_brute_force(seed):
    """Random sparse graphs with many leaves: pruned = degree one and not the
    smaller end of an isolated edge; the pruned graph is the induced subgraph
    on the kept vertices, relabelled in ascending order."""
    g = inputs.random_tree_plus_edges(300, 40, seed)
    h = inputs.to_csr(310, np.concatenate([g.edges()[:, 0], [300, 302, 305]]),
                      np.concatenate([g.edges()[:, 1], [301, 303, 306]]))
    A = _dense(h)
    deg = A.sum(1)
    pr = oracle.prune(h.n, h.row_ptr, h.col_idx)
    pruned = np.zeros(h.n, dtype=bool)
    for v in range(h.n):
        if deg[v] == 1:
            w = int(np.flatnonzero(A[v])[0])
            pruned[v] = not (deg[w] == 1 and w > v)
    assert np.array_equal(pr.anchor >= 0, pruned)
    for v in np.flatnonzero(pruned):
        assert A[v, pr.anchor[v]] and pr.anchor[pr.anchor[v]] == -1
    assert pr.leaves.sum() == pruned.sum()
    np.testing.assert_array_equal(np.bincount(pr.anchor[pruned], minlength=h.n), pr.leaves)
    kept = np.flatnonzero(~pruned)
    assert pr.n == kept.size
    assert np.array_equal(pr.new_id[kept], np.arange(kept.size))
    sub = A[np.ix_(kept, kept)]
    got = np.zeros_like(sub)
    for v in range(pr.n):
        got[v, pr.col_idx[pr.row_ptr[v]:pr.row_ptr[v + 1]]] = True
        assert np.all(np.diff(pr.col_idx[pr.row_ptr[v]:pr.row_ptr[v + 1]]) > 0)
    assert np.array_equal(got, sub)


# ----------------------------------------------------- leaf-weighted repulsion

@pytest.mark.parametrize("m0,m1", [(1.0, 1.0), (3.0, 1.0), (1.0, 5.0), (2.0, 7.0)])
def test_weighted_two_vertices_closed_form(m0, m1):
    """Edge of length delta: v feels m_u d^2/delta outwards from u and
    delta^2/d inwards (attraction is not weighted)."""
    d, delta = 10.0, 4.0
    g = inputs.path_graph(2)
    pos = np.array([[0.0, 0.0], [delta, 0.0]])
    kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, 2)
    F, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, d, pos, mass=[m0, m1])
    np.testing.assert_allclose(F[1], [m0 * d * d / delta - delta * delta / d, 0.0], rtol=1e-13)
    np.testing.assert_allclose(F[0], [-(m1 * d * d / delta - delta * delta / d), 0.0],
                               rtol=1e-13)


def test_unit_mass_is_unweighted():
    g = inputs.barabasi_albert(200, 2, 5)
    pos = inputs.uniform_positions(g.n, 9, 300.0, 300.0).astype(np.float64)
    kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, 2)
    F0, c0 = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 30.0, pos)
    F1, c1 = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 30.0, pos, mass=np.ones(g.n))
    assert np.array_equal(F0, F1) and c0 == c1


@pytest.mark.parametrize("k", [1, 2, 3])
def test_weighted_action_reaction(k):
    """N_v(k) is symmetric, so the weighted repulsions cancel:
    sum_v m_v F^rep_v = 0 (F^rep = F minus the attraction-only force)."""
    g = inputs.random_tree_plus_edges(150, 30, 11)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    m = pr.mass()
    assert m.max() > 2
    pos = inputs.uniform_positions(pr.n, 4, 200.0, 200.0).astype(np.float64)
    kp, ki = oracle.khop(pr.n, pr.row_ptr, pr.col_idx, k)
    F, _ = oracle.forces(pr.n, pr.row_ptr, pr.col_idx, kp, ki, 25.0, pos, mass=m)
    Fa, _ = oracle.forces(pr.n, pr.row_ptr, pr.col_idx, np.zeros(pr.n + 1, np.int64),
                          np.zeros(0, np.int32), 25.0, pos, mass=m)
    rep = F - Fa
    scale = np.abs(m[:, None] * rep).sum()
    assert np.abs((m[:, None] * rep).sum(0)).max() <= 1e-12 * scale
    # the attraction alone sums to zero without weights
    assert np.abs(Fa.sum(0)).max() <= 1e-12 * np.abs(Fa).sum()


def test_weighted_linear_in_mass():
    """F_v(m) = A_v + sum_u m_u R_vu: doubling (m - 1) doubles F(m) - F(1)."""
    g = inputs.barabasi_albert(120, 2, 8)
    pos = inputs.uniform_positions(g.n, 3, 150.0, 150.0).astype(np.float64)
    kp, ki = oracle.khop(g.n, g.row_ptr, g.col_idx, 2)
    rng = np.random.default_rng(0)
    extra = rng.integers(0, 5, g.n).astype(np.float64)
    F1, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 20.0, pos)
    Fa, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 20.0, pos, mass=1 + extra)
    Fb, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, kp, ki, 20.0, pos, mass=1 + 2 * extra)
    np.testing.assert_allclose(Fb - F1, 2 * (Fa - F1), rtol=1e-9, atol=1e-9 * np.abs(Fb).max())


def test_weighted_step_and_layout_use_mass():
    g = inputs.random_tree_plus_edges(80, 20, 2)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    m = pr.mass()
    pos = inputs.uniform_positions(pr.n, 5, 100.0, 100.0).astype(np.float64)
    kp, ki = oracle.khop(pr.n, pr.row_ptr, pr.col_idx, 2)
    F, _ = oracle.forces(pr.n, pr.row_ptr, pr.col_idx, kp, ki, 15.0, pos, mass=m)
    x1, F1, D1, _ = oracle.step(pr.n, pr.row_ptr, pr.col_idx, kp, ki, 15.0, 3.0, pos, mass=m)
    assert np.array_equal(F, F1)
    np.testing.assert_array_equal(x1, pos + oracle.cap(F, 3.0))
    temps = np.array([3.0, 2.0])
    xl, run, _ = oracle.layout(pr.n, pr.row_ptr, pr.col_idx, kp, ki, 15.0, temps, pos, mass=m)
    x2, _, _, _ = oracle.step(pr.n, pr.row_ptr, pr.col_idx, kp, ki, 15.0, 2.0, x1, mass=m)
    assert run == 2 and np.array_equal(xl, x2)


# ---------------------------------------------------------------- reinsertion

def test_reinsert_star_uniform_circle():
    """Centre without incident edges: radius 0.2 d, leaves at angles 2 pi j/L
    in ascending id."""
    d = 30.0
    g = inputs.star_graph(4)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    out = oracle.reinsert(pr, d, np.array([[5.0, -2.0]]))
    np.testing.assert_array_equal(out[0], [5.0, -2.0])
    for j in range(4):
        th = 2 * math.pi * j / 4
        np.testing.assert_allclose(out[1 + j], [5.0 + 6.0 * math.cos(th), -2.0 + 6.0 * math.sin(th)],
                                   rtol=0, atol=1e-12)


def test_reinsert_isolated_edge():
    g = inputs.path_graph(2)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    out = oracle.reinsert(pr, 10.0, np.array([[1.0, 1.0]]))
    np.testing.assert_allclose(out, [[1.0, 1.0], [3.0, 1.0]], atol=1e-12)


def test_reinsert_opposite_the_bisector():
    """Triangle 0-1-2 with one leaf (3) on vertex 0; edges leave 0 at angles
    0 and pi/2, so the leaf goes to 5 pi / 4, at 0.2 of the shorter edge."""
    g = inputs.to_csr(4, [0, 1, 2, 0], [1, 2, 0, 3])
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    assert pr.n == 3 and list(pr.leaves) == [1, 0, 0, 0]
    pos = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 15.0]])
    out = oracle.reinsert(pr, 99.0, pos)
    np.testing.assert_array_equal(out[:3], pos)
    np.testing.assert_allclose(out[3], [-math.sqrt(2.0), -math.sqrt(2.0)], atol=1e-12)


def test_reinsert_two_leaves_between_collinear_edges():
    """Square 0-1-2-3 with leaves 4, 5 on 0; the edges leave 0 at 0 and pi, so
    the leaves go to pi/2 and 3 pi/2 at radius 0.2 * 5."""
    g = inputs.to_csr(6, [0, 1, 2, 3, 0, 0], [1, 2, 3, 0, 4, 5])
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    pos = np.array([[0.0, 0.0], [5.0, 0.0], [5.0, 9.0], [-5.0, 0.0]])
    out = oracle.reinsert(pr, 99.0, pos)
    np.testing.assert_allclose(out[4], [0.0, 1.0], atol=1e-12)
    np.testing.assert_allclose(out[5], [0.0, -1.0], atol=1e-12)


def _ang_dist(a, b):
    x = np.abs(a - b) % (2 * math.pi)
    return np.minimum(x, 2 * math.pi - x)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_reinsert_rotation_is_optimal(seed):
    """Random drawing: every leaf sits at 0.2 x the shortest incident edge,
    the leaves of a vertex are 2 pi / L apart, and their smallest angular
    distance to the incident edges is the best any rotation achieves (grid
    search over the rotation)."""
    g = inputs.random_tree_plus_edges(200, 60, seed)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    pos = inputs.uniform_positions(pr.n, seed + 10, 500.0, 500.0).astype(np.float64)
    d = 40.0
    out = oracle.reinsert(pr, d, pos)
    kept = np.flatnonzero(pr.new_id >= 0)
    np.testing.assert_array_equal(out[kept], pos[pr.new_id[kept]])
    grid = np.linspace(0.0, 2 * math.pi, 20001)
    checked = 0
    for v in kept:
        L = pr.leaves[v]
        if L == 0:
            continue
        i = pr.new_id[v]
        nb = pr.col_idx[pr.row_ptr[i]:pr.row_ptr[i + 1]]
        vec = pos[nb] - pos[i]
        lens = np.hypot(vec[:, 0], vec[:, 1])
        rho = 0.2 * (lens.min() if nb.size else d)
        leaves = np.flatnonzero(pr.anchor == v)
        rel = out[leaves] - pos[i]
        np.testing.assert_allclose(np.hypot(rel[:, 0], rel[:, 1]), rho, rtol=1e-12)
        th = np.arctan2(rel[:, 1], rel[:, 0])
        steps = (th - th[0]) % (2 * math.pi)
        np.testing.assert_allclose(np.sort(steps), 2 * math.pi * np.arange(L) / L, atol=1e-9)
        if nb.size == 0:
            continue
        edge_ang = np.arctan2(vec[:, 1], vec[:, 0])
        got = _ang_dist(th[:, None], edge_ang[None, :]).min()
        cand = grid[:, None] + 2 * math.pi * np.arange(L)[None, :] / L
        best = _ang_dist(cand[:, :, None], edge_ang[None, None, :]).min(axis=(1, 2)).max()
        assert got >= best - 1e-3
        checked += 1
    assert checked > 10
