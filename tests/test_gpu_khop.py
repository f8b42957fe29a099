"""GPU parity of the k-hop lists N_v(k) (Section 4.5): bit-exact against the
oracle's BFS, on small graphs of every family and at the full benchmark sizes
(every row of R-MAT 18 and Barabasi-Albert 100k, compared in chunks)."""
import ctypes

import numpy as np
import pytest

from gpu_common import oracle_rows, require_gpu, small_graph_suite
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _build(G, g, k):
    rp, ci = G.to_device_csr(g)
    return G.build_khop(rp, ci, k)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_small_graphs_bit_exact(G, k):
    for g in small_graph_suite():
        if k == 4 and g.n > 3000:
            continue
        print(f"khop {g.name} n={g.n} k={k}", flush=True)
        kh = _build(G, g, k)
        ptr, idx = kh.export()
        optr, oidx = oracle_rows(g, k)
        assert np.array_equal(ptr, optr), g.name
        assert np.array_equal(idx, oidx), g.name
        inf = kh.info()
        assert inf["total_pairs"] == int(optr[-1])
        assert inf["n_active"] == int((np.diff(g.row_ptr) > 0).sum())
        kh.free()


@pytest.mark.parametrize("k", [2, 3])
def test_global_bitmap_path_bit_exact(G, k, monkeypatch):
    """The frontier expansion with its bitmap in global memory (the path of
    graphs too large for an LDS bitmap), forced on graphs of every family:
    the same rows as the oracle."""
    monkeypatch.setenv("GILA_BFS_BITMAP", "global")
    for g in small_graph_suite():
        if g.n > 5000:
            continue
        kh = _build(G, g, k)
        ptr, idx = kh.export()
        optr, oidx = oracle_rows(g, k)
        assert np.array_equal(ptr, optr), g.name
        assert np.array_equal(idx, oidx), g.name
        kh.free()


def test_repeated_builds_with_queued_frontiers(G):
    """k >= 3 records each level's new vertices in a per-workgroup queue that
    the next level expands; repeated builds of graphs with many short and some
    long frontier rows give the oracle's rows every time."""
    cases = [(inputs.barabasi_albert(20000, 3, seed=41), 3),
             (inputs.watts_strogatz(20000, 6, 0.1, seed=42), 4)]
    for g, k in cases:
        optr, oidx = oracle_rows(g, k)
        for rep in range(4):
            kh = _build(G, g, k)
            ptr, idx = kh.export()
            assert np.array_equal(ptr, optr), (g.name, k, rep)
            assert np.array_equal(idx, oidx), (g.name, k, rep)
            kh.free()


def test_freed_handles_reuse_and_return_cached_memory(G):
    """A freed handle's device blocks stay in the library's cache: a rebuild of
    the same graph reuses them and gives the same rows, and releasing the cache
    returns them to the device (a second release finds nothing)."""
    g = inputs.barabasi_albert(20000, 3, seed=43)
    G.release_cached_memory()
    kh = _build(G, g, 2)
    ptr0, idx0 = kh.export()
    kh.free()
    kh = _build(G, g, 2)
    ptr1, idx1 = kh.export()
    kh.free()
    assert np.array_equal(ptr0, ptr1) and np.array_equal(idx0, idx1)
    assert G.release_cached_memory() > 0
    assert G.release_cached_memory() == 0


def _expected_order(g, counts):
    """The internal order rule written out with numpy sorts: the caller's
    order (hub rows of >= 8192 entries first) when >= 70% of the adjacency
    entries join ids less than 1024 apart, else |N_v(k)| descending; isolated
    vertices last; ties by ascending caller id."""
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    near = int((np.abs(g.col_idx.astype(np.int64) - src) < 1024).sum())
    caller = g.col_idx.size > 0 and near >= 0.7 * g.col_idx.size
    iso = deg == 0
    if caller:
        key = np.where(iso, 2, np.where(counts >= 8192, 0, 1))
    else:
        key = np.where(iso, g.n, g.n - 1 - counts)
    return np.lexsort((np.arange(g.n), key)).astype(np.int32), caller


def test_internal_order_follows_the_rule(G):
    """The device-built internal order equals the rule computed on the host
    from the exported list lengths, for degree-ordered graphs (R-MAT with
    isolated vertices, Barabasi-Albert), a caller-ordered mesh, and a ring
    with a far-connected hub (caller order with a hub row first)."""
    ring_n, hub_deg = 20000, 3500
    rng = np.random.default_rng(5)
    hub = ring_n // 2
    others = np.delete(np.arange(ring_n), hub)
    spokes = np.sort(rng.choice(others, hub_deg, replace=False))
    u = np.concatenate([np.arange(ring_n), np.full(hub_deg, hub, np.int64)])
    v = np.concatenate([(np.arange(ring_n) + 1) % ring_n, spokes])
    ring_hub = inputs.to_csr(ring_n, u, v, name="ring_hub")
    cases = [(inputs.rmat(14, 4, 0.57, 0.19, 0.19, seed=3), 2, False),
             (inputs.barabasi_albert(5000, 3, seed=9), 3, False),
             (inputs.grid_graph(60, 70), 2, True),
             (ring_hub, 2, True)]
    for g, k, want_caller in cases:
        kh = _build(G, g, k)
        ptr, _ = kh.export()
        want, caller = _expected_order(g, np.diff(ptr))
        assert caller == want_caller, g.name
        assert np.array_equal(kh.order(), want), g.name
        kh.free()
    assert np.diff(inputs.rmat(14, 4, 0.57, 0.19, 0.19, seed=3).row_ptr).min() == 0
    kh = _build(G, ring_hub, 2)
    assert kh.order()[0] == hub  # the hub (|N(2)| >= 8192) leads
    kh.free()


def test_grid32_config_total(G):
    g = inputs.grid_graph(32, 32)
    kh = _build(G, g, 2)
    assert kh.info()["total_pairs"] == 11652


def test_empty_and_degenerate_graphs(G):
    for g in (inputs.to_csr(0, [], []), inputs.to_csr(1, [], []), inputs.to_csr(7, [], []),
              inputs.path_graph(2)):
        for k in (1, 3):
            if g.n == 0:
                import torch
                rp = torch.zeros(1, dtype=torch.int64, device="cuda")
                ci = torch.zeros(0, dtype=torch.int32, device="cuda")
                kh = G.build_khop(rp, ci, k)
            else:
                kh = _build(G, g, k)
            ptr, idx = kh.export()
            optr, oidx = oracle_rows(g, k)
            assert np.array_equal(ptr, optr) and np.array_equal(idx, oidx)


def _bad_csr(G, rp, ci, k=2):
    import torch
    rpd = torch.tensor(rp, dtype=torch.int64, device="cuda")
    cid = torch.tensor(ci, dtype=torch.int32, device="cuda")
    with pytest.raises(G.GilaError) as e:
        G.build_khop(rpd, cid, k)
    assert e.value.code == G.GILA_EINVAL
    return str(e.value)


def test_malformed_csr_rejected(G):
    assert "not symmetric" in _bad_csr(G, [0, 1, 2, 2], [1, 2])             # 0->1, 1->2 only
    assert "self-loop" in _bad_csr(G, [0, 2, 4, 4], [0, 1, 0, 1])
    assert "ascending" in _bad_csr(G, [0, 2, 3, 4], [2, 1, 0, 0])
    assert "out of range" in _bad_csr(G, [0, 1, 2], [5, 0])
    _bad_csr(G, [0, 2, 1], [1, 0])                                           # non-monotone
    _bad_csr(G, [1, 2, 2], [1, 0])                                           # row_ptr[0] != 0
    with pytest.raises(G.GilaError):
        _build(G, inputs.path_graph(4), 0)


@pytest.mark.parametrize("which", ["ba100k_k3", "rmat18_k2"])
def test_full_size_lists(G, which):
    """Full benchmark graphs: every row compared with the oracle's BFS, bit
    for bit, in chunks of at most ~24M entries (P is ~0.25 G and ~0.5 G)."""
    if which == "ba100k_k3":
        g, k = inputs.barabasi_albert(100000, 3, seed=2), 3
    else:
        g, k = inputs.rmat(18, 4, 0.57, 0.19, 0.19, seed=3), 2
    print(f"full-size khop {which}", flush=True)
    kh = _build(G, g, k)
    all_v = np.arange(g.n, dtype=np.int32)
    # exact sizes of every row (oracle count pass over all vertices)
    import oracle
    sizes = np.zeros(g.n, dtype=np.int64)
    lib = oracle._load()
    rc = lib.orc_khop_count(g.n, g.row_ptr, g.col_idx, k, g.n, None, sizes)
    assert rc == 0
    gptr = np.zeros(g.n + 1, dtype=np.int64)
    L = G.lib()
    assert L.gila_khop_export_rows(kh.handle, g.n, all_v.ctypes.data, gptr.ctypes.data,
                                   None) == 0
    assert np.array_equal(np.diff(gptr), sizes)
    assert kh.info()["total_pairs"] == int(sizes.sum())
    # every row, chunk by chunk
    cum = np.concatenate([[0], np.cumsum(sizes)])
    limit = 24 << 20
    lo, chunks, checked = 0, 0, 0
    while lo < g.n:
        hi = int(np.searchsorted(cum, cum[lo] + limit, side="right")) - 1
        hi = min(max(hi, lo + 1), g.n)
        verts = all_v[lo:hi]
        sp, si = kh.export_rows(verts)
        op, oi = oracle_rows(g, k, verts=verts)
        assert np.array_equal(sp, op), (lo, hi)
        assert np.array_equal(si, oi), (lo, hi)
        checked += int(op[-1])
        chunks += 1
        if chunks % 8 == 0:
            print(f"  {which}: rows [0, {hi}) equal ({checked} entries)", flush=True)
        lo = hi
    assert checked == int(sizes.sum())
    print(f"{which}: all {g.n} rows, {checked} entries bit-exact", flush=True)


def test_build_is_deterministic(G):
    g = inputs.barabasi_albert(5000, 3, seed=9)
    a = _build(G, g, 3).export()
    b = _build(G, g, 3).export()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
