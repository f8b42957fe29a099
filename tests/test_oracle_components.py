"""Pins of the oracle's connected components, matrix packing and
per-component layout (Sections 4.6 and 5.1).

Components are checked against scipy's connected_components (an independent
library routine) and hand cases; packing against a hand-computed matrix and
its invariants (translation only, disjoint cells, order by size); the
per-component driver against the plain layout of each component with the cap
of its own size and aspect ratio, and its halting rule per component.
"""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from paper_1606_02162_amd import inputs


def _union(*graphs):
    us, vs, off = [], [], 0
    for g in graphs:
        e = g.edges()
        us.append(e[:, 0] + off)
        vs.append(e[:, 1] + off)
        off += g.n
    return inputs.to_csr(off, np.concatenate(us), np.concatenate(vs))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_components_against_scipy(seed):
    rng = np.random.default_rng(seed)
    n = 2000
    m = 900
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    keep = u != v
    g = inputs.to_csr(n, u[keep], v[keep])
    label, count = oracle.components(g.n, g.row_ptr, g.col_idx)
    A = csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(n, n))
    nc, lab = connected_components(A, directed=False)
    assert count == nc
    minid = np.full(nc, n)
    np.minimum.at(minid, lab, np.arange(n))
    assert np.array_equal(label, minid[lab])


def test_components_hand_cases():
    g = inputs.to_csr(7, [1, 2, 5], [2, 3, 6])   # {0}, {1,2,3}, {4}, {5,6}
    label, count = oracle.components(g.n, g.row_ptr, g.col_idx)
    assert count == 4 and list(label) == [0, 1, 1, 1, 4, 5, 5]
    p = inputs.path_graph(50)
    label, count = oracle.components(p.n, p.row_ptr, p.col_idx)
    assert count == 1 and not label.any()
    e = inputs.to_csr(0, [], [])
    label, count = oracle.components(0, e.row_ptr, e.col_idx)
    assert count == 0 and label.size == 0


def test_pack_hand_computed():
    """Components {0,1,2} (size 3), {3,4}, {5,6} (size 2), {7} (size 1):
    ceil(sqrt(4)) = 2 columns.  Ranks: {0,1,2} (0,0), {3,4} (0,1), {5,6}
    (1,0), {7} (1,1)."""
    label = np.array([0, 0, 0, 3, 3, 5, 5, 7], dtype=np.int32)
    pos = np.array([[10, 10], [14, 10], [12, 13],   # box 4 x 3 from (10, 10)
                    [-5, -5], [-5, 1],              # box 0 x 6 from (-5, -5)
                    [100, 100], [102, 101],         # box 2 x 1 from (100, 100)
                    [7, 7]], dtype=np.float64)      # box 0 x 0
    gap = 1.5
    out = oracle.pack(label, gap, pos)
    # column widths max(4, 2) = 4 and max(0, 0) = 0; row heights max(3, 6) = 6, max(1, 0) = 1
    colx = [0.0, 4.0 + gap]
    rowy = [0.0, 6.0 + gap]
    exp = np.array([[colx[0] + 0, rowy[0] + 0], [colx[0] + 4, rowy[0] + 0], [colx[0] + 2, rowy[0] + 3],
                    [colx[1] + 0, rowy[0] + 0], [colx[1] + 0, rowy[0] + 6],
                    [colx[0] + 0, rowy[1] + 0], [colx[0] + 2, rowy[1] + 1],
                    [colx[1] + 0, rowy[1] + 0]])
    np.testing.assert_array_equal(out, exp)


@pytest.mark.parametrize("seed", [4, 5])
def test_pack_invariants(seed):
    rng = np.random.default_rng(seed)
    g = _union(*[inputs.random_tree_plus_edges(int(s), 2, seed=int(s) + seed)
                 for s in rng.integers(3, 40, 23)], inputs.to_csr(5, [], []))
    label, count = oracle.components(g.n, g.row_ptr, g.col_idx)
    pos = rng.uniform(-500, 500, (g.n, 2))
    out = oracle.pack(label, 10.0, pos)
    roots = np.flatnonzero(label == np.arange(g.n))
    sizes = np.array([(label == r).sum() for r in roots])
    boxes = {}
    for r in roots:
        vs = label == r
        d = out[vs] - pos[vs]
        # a pure translation of the component
        np.testing.assert_allclose(d, d[0][None, :].repeat(vs.sum(), 0), rtol=0, atol=1e-9)
        boxes[r] = (out[vs].min(0), out[vs].max(0))
        assert np.all(out[vs].min(0) >= -1e-9)
    # cells do not overlap: any two boxes are separated by at least the gap on one axis
    rs = list(roots)
    for i in range(len(rs)):
        for j in range(i + 1, len(rs)):
            (a0, a1), (b0, b1) = boxes[rs[i]], boxes[rs[j]]
            sep = max(b0[0] - a1[0], a0[0] - b1[0], b0[1] - a1[1], a0[1] - b1[1])
            assert sep >= 10.0 - 1e-9
    # the largest component sits in the first cell (lower-left corner at the origin)
    big = roots[np.argmax(sizes)]
    np.testing.assert_allclose(boxes[big][0], [0.0, 0.0], atol=1e-9)
    assert count == roots.size


def test_component_aspect():
    x = np.array([[0.0, 0.0], [100.0, 50.0], [30.0, 10.0]])
    assert oracle.component_aspect(x) == 0.5
    assert oracle.component_aspect(np.array([[1.0, 2.0], [5.0, 2.0]])) == 1.0


def test_layout_components_is_each_component_alone():
    """Each component is the plain layout of its own subgraph with the cap
    sqrt((n_C / a_C) d) 0.93^h, then the drawings are packed."""
    a = inputs.random_tree_plus_edges(60, 20, seed=1)
    b = inputs.grid_graph(5, 7)
    g = _union(a, b, inputs.to_csr(2, [], []))
    d, k, H = 12.0, 2, 15
    pos = inputs.uniform_positions(g.n, seed=3, width=300.0, height=200.0).astype(np.float64)
    out, label, runs = oracle.layout_components(g.n, g.row_ptr, g.col_idx, k, d, H, pos,
                                                stop_fraction=0.0)
    expect = pos.copy()
    for verts, sub in ((np.arange(a.n), a), (a.n + np.arange(b.n), b)):
        x0 = pos[verts]
        w, h = np.ptp(x0[:, 0]), np.ptp(x0[:, 1])
        temps = math.sqrt(verts.size / (h / w) * d) * 0.93 ** np.arange(H)
        kp, ki = oracle.khop(sub.n, sub.row_ptr, sub.col_idx, k)
        xf, run, _ = oracle.layout(sub.n, sub.row_ptr, sub.col_idx, kp, ki, d, temps, x0)
        expect[verts] = xf
        assert runs[int(verts[0])] == H
    np.testing.assert_allclose(out, oracle.pack(label, d, expect), rtol=0, atol=1e-9)


def test_halting_is_per_component():
    """An edge drawn at its equilibrium length d stops after one iteration,
    while a larger component keeps going."""
    d = 10.0
    g = _union(inputs.path_graph(2), inputs.random_tree_plus_edges(80, 40, seed=2))
    pos = inputs.uniform_positions(g.n, seed=4, width=400.0, height=400.0).astype(np.float64)
    pos[1] = pos[0] + np.array([d * 0.6, d * 0.8])
    out, label, runs = oracle.layout_components(g.n, g.row_ptr, g.col_idx, 2, d, 30, pos,
                                                stop_fraction=0.15, stop_displacement=0.01)
    assert runs[0] == 1
    assert runs[2] > 1
