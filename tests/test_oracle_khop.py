"""Pins of the oracle's k-neighbourhoods N_v(k) (Section 4.5).

The oracle computes N_v(k) by one BFS per vertex.  It is pinned here against
things that do not share its code:
  * brute-force all-pairs distances (Floyd-Warshall on tiny graphs);
  * an independent simulation of the paper's controlled flooding with TTL
    (Section 4.5: first superstep sends (position, id, TTL = k); second
    superstep processes, records the sender in H_v, decrements and forwards;
    later supersteps skip senders already in H_v, else record, decrement and
    forward while TTL > 0);
  * closed-form sizes on grids, cycles, stars, complete graphs;
  * symmetry (u in N_v(k) iff v in N_u(k)) and monotonicity in k.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1606_02162_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(ptr, idx):
    return [idx[ptr[i]:ptr[i + 1]].tolist() for i in range(len(ptr) - 1)]


def _floyd(g):
    n = g.n
    inf = 10 ** 9
    dist = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(dist, 0)
    e = g.edges()
    dist[e[:, 0], e[:, 1]] = 1
    dist[e[:, 1], e[:, 0]] = 1
    for w in range(n):
        dist = np.minimum(dist, dist[:, [w]] + dist[[w], :])
    return dist


def _ttl_flood(g, k, self_in_h=True):
    """Literal superstep simulation of the flooding of Section 4.5.

    Returns, for every vertex v, the set of origins whose message v used for
    a force (the contents of H_v at the end of the iteration, minus v).
    ``self_in_h`` is the reading that H_v starts out holding v, so a message
    returning to its origin is discarded.
    """
    n = g.n
    adj = [g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() for v in range(n)]
    H = [set([v]) if self_in_h else set() for v in range(n)]
    used = [set() for _ in range(n)]
    # superstep 1: every vertex sends (id, TTL=k) to its neighbours
    inbox = [[] for _ in range(n)]
    for v in range(n):
        for w in adj[v]:
            inbox[w].append((v, k))
    # superstep 2: process every message, record, decrement, forward all
    outbox = [[] for _ in range(n)]
    for v in range(n):
        for origin, ttl in inbox[v]:
            # every second-superstep message comes from a distinct neighbour
            used[v].add(origin)
            H[v].add(origin)
            for w in adj[v]:
                outbox[w].append((origin, ttl - 1))
    inbox = outbox
    # supersteps i > 2
    while any(inbox):
        outbox = [[] for _ in range(n)]
        for v in range(n):
            for origin, ttl in inbox[v]:
                if origin in H[v]:
                    continue
                used[v].add(origin)
                H[v].add(origin)
                ttl -= 1
                if ttl > 0:
                    for w in adj[v]:
                        outbox[w].append((origin, ttl))
        inbox = outbox
    return [sorted(s - {v}) for v, s in enumerate(used)]


def _random_small_graphs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(2, 26))
        m = int(rng.integers(1, min(n * (n - 1) // 2, 3 * n) + 1))
        out.append(inputs.erdos_renyi(n, m, seed=seed * 1000 + i))
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_khop_equals_bruteforce_distances(k):
    for g in _random_small_graphs(40, seed=11 + k):
        dist = _floyd(g)
        ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
        for v, row in enumerate(_rows(ptr, idx)):
            expect = [u for u in range(g.n) if u != v and dist[v, u] <= k]
            assert row == expect, (g.name, k, v)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_khop_equals_literal_ttl_flooding(k):
    """For k >= 2 the paper's flooding delivers exactly the radius-k ball."""
    for g in _random_small_graphs(30, seed=97 + k):
        ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
        assert _rows(ptr, idx) == _ttl_flood(g, k), (g.name, k)


def test_k1_literal_flooding_reaches_distance_two_reading():
    """With k = 1 the literal text forwards every message in the second
    superstep, so it reaches distance 2.  The library reads k = 1 as the
    radius-1 ball of the definition in Section 4.5; this test records the gap."""
    g = inputs.path_graph(5)
    flood = _ttl_flood(g, 1)
    assert flood[0] == [1, 2]
    ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, 1)
    assert _rows(ptr, idx)[0] == [1]


def test_khop_closed_form_sizes():
    # grid interior vertex: |N_v(k)| = 2k(k+1)
    g = inputs.grid_graph(15, 15)
    centre = 7 * 15 + 7
    for k in range(1, 6):
        ptr, _ = oracle.khop(g.n, g.row_ptr, g.col_idx, k, verts=[centre])
        assert ptr[1] == 2 * k * (k + 1)
    # cycle: min(2k, n-1)
    for n in (3, 4, 7, 10):
        g = inputs.cycle_graph(n)
        for k in range(1, 7):
            ptr, _ = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
            assert np.all(np.diff(ptr) == min(2 * k, n - 1))
    # star K_{1,m}: hub sees m for every k; a leaf sees 1 for k = 1, m for k >= 2
    g = inputs.star_graph(9)
    for k in range(1, 4):
        ptr, _ = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
        sizes = np.diff(ptr)
        assert sizes[0] == 9
        assert np.all(sizes[1:] == (1 if k == 1 else 9))
    # complete graph: n - 1
    g = inputs.complete_graph(8)
    ptr, _ = oracle.khop(g.n, g.row_ptr, g.col_idx, 1)
    assert np.all(np.diff(ptr) == 7)


def test_grid32_totals_golden():
    """Total ordered pairs of the 32x32 grid, counted in closed form."""
    with open(os.path.join(GOLDEN, "grid32_khop_totals.json")) as f:
        gold = json.load(f)
    g = inputs.grid_graph(32, 32)
    for k_str, total in gold["totals"].items():
        ptr, _ = oracle.khop(g.n, g.row_ptr, g.col_idx, int(k_str))
        assert int(ptr[-1]) == total


def test_khop_symmetric_and_monotone():
    g = inputs.barabasi_albert(400, 2, seed=5)
    prev = None
    for k in (1, 2, 3):
        ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
        rows = _rows(ptr, idx)
        pairs = {(v, u) for v, r in enumerate(rows) for u in r}
        assert all((u, v) in pairs for (v, u) in pairs)
        assert all(v not in r for v, r in enumerate(rows))
        if prev is not None:
            assert all(set(p) <= set(r) for p, r in zip(prev, rows))
        if k == 1:
            assert rows == _rows(g.row_ptr, g.col_idx)
        prev = rows


def test_khop_subset_rows_match_full():
    g = inputs.rmat(10, 4, 0.57, 0.19, 0.19, seed=3)
    ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, 2)
    verts = np.array([0, 5, 17, 1023, 400, 5], dtype=np.int32)
    sptr, sidx = oracle.khop(g.n, g.row_ptr, g.col_idx, 2, verts=verts)
    full = _rows(ptr, idx)
    for i, v in enumerate(verts):
        assert sidx[sptr[i]:sptr[i + 1]].tolist() == full[v]


def test_khop_isolated_and_empty():
    g = inputs.to_csr(5, [0], [1])
    ptr, idx = oracle.khop(g.n, g.row_ptr, g.col_idx, 3)
    assert np.diff(ptr).tolist() == [1, 1, 0, 0, 0]
    g0 = inputs.to_csr(0, [], [])
    ptr, idx = oracle.khop(0, g0.row_ptr, g0.col_idx, 2)
    assert ptr.tolist() == [0] and idx.size == 0
