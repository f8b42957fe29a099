"""Seeded input generators: canonical CSR, exact sizes, determinism, and the
SplitMix64 counter-based placement against its published output values."""
import json
import os

import numpy as np
import pytest

from paper_1606_02162_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _canonical(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp.dtype == np.int64 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == ci.size and np.all(np.diff(rp) >= 0)
    for v in range(g.n):
        row = ci[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
        assert not np.any(row == v)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((b, a) in fwd for (a, b) in fwd)


def test_splitmix64_published_values():
    with open(os.path.join(GOLDEN, "splitmix64_vectors.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        got = inputs.splitmix64_u64(case["seed"], np.arange(len(case["outputs"])))
        assert [int(x) for x in got] == [int(x, 16) for x in case["outputs"]]


def test_uniform_positions_range_and_determinism():
    p = inputs.uniform_positions(10000, seed=0, width=1000.0, height=500.0)
    assert p.shape == (10000, 2)
    assert p[:, 0].min() >= 0 and p[:, 0].max() < 1000
    assert p[:, 1].min() >= 0 and p[:, 1].max() < 500
    assert np.array_equal(p, inputs.uniform_positions(10000, seed=0, width=1000.0, height=500.0))
    assert not np.array_equal(p, inputs.uniform_positions(10000, seed=1, width=1000.0,
                                                          height=500.0))
    # counters 2v / 2v+1: prefix property
    q = inputs.uniform_positions(100, seed=0, width=1000.0, height=500.0)
    assert np.array_equal(q, p[:100])
    assert abs(p[:, 0].mean() - 500) < 10


def test_grid_exact():
    g = inputs.grid_graph(32, 32)
    assert g.n == 1024 and g.m == 1984
    _canonical(g)
    deg = g.degrees()
    assert sorted(set(deg.tolist())) == [2, 3, 4] and (deg == 2).sum() == 4


def test_small_families():
    for g, m in [(inputs.path_graph(7), 6), (inputs.cycle_graph(9), 9), (inputs.star_graph(5), 5),
                 (inputs.complete_graph(6), 15)]:
        _canonical(g)
        assert g.m == m


def test_to_csr_drops_loops_and_duplicates():
    g = inputs.to_csr(4, [0, 0, 1, 2, 2, 3], [1, 1, 0, 2, 3, 2])
    assert g.m == 2
    _canonical(g)


def test_barabasi_albert_shape():
    g = inputs.barabasi_albert(3000, 3, seed=2)
    _canonical(g)
    assert g.m == 3 + (3000 - 4) * 3
    deg = g.degrees()
    assert deg.min() >= 3 and deg.max() > 60          # heavy tail
    g2 = inputs.barabasi_albert(3000, 3, seed=2)
    assert np.array_equal(g.col_idx, g2.col_idx)


def test_rmat_shape():
    g = inputs.rmat(12, 4, 0.57, 0.19, 0.19, seed=3)
    _canonical(g)
    assert g.n == 4096 and 0.8 * 4 * 4096 < g.m <= 4 * 4096
    assert (g.degrees() == 0).sum() > 0


def test_tree_plus_edges_connected():
    g = inputs.random_tree_plus_edges(500, 250, seed=4)
    _canonical(g)
    assert g.m == 499 + 250
    seen = {0}
    stack = [0]
    while stack:
        v = stack.pop()
        for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist():
            if u not in seen:
                seen.add(u)
                stack.append(u)
    assert len(seen) == 500


def test_watts_strogatz_shape():
    g = inputs.watts_strogatz(1000, 6, 0.1, seed=5)
    _canonical(g)
    assert g.m == 3000
    lattice = inputs.watts_strogatz(1000, 6, 0.0, seed=5)
    assert np.all(lattice.degrees() == 6)


def test_erdos_renyi_exact_m():
    g = inputs.erdos_renyi(1000, 2500, seed=1)
    _canonical(g)
    assert g.m == 2500


def test_log_uniform_and_poisson():
    s = inputs.log_uniform_sizes(4096, 50, 5000, seed=4)
    assert s.min() >= 50 and s.max() < 5000
    t = inputs.poisson_arrivals(2000, 200.0, seed=5)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 2000 - 1 / 200) < 0.001
