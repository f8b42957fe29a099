"""GPU parity of pruning, leaf-weighted repulsion and reinsertion against the
FP64 oracle (Sections 4.3 and 4.6).

  * pruning: anchors, leaf counts, new ids and the pruned graph bit-exact;
  * weighted forces: one step of the pruned graph with each kept vertex's
    repulsion weighted by 1 + its leaves (and with arbitrary weights), on the
    segment and direct paths, to the layout gates (FP32 e_F, e_x <= 1e-5;
    FP64 1e-12);
  * reinsertion: every position against the oracle's from the same kept
    drawing, where the widest angular gap is unique; where two gaps tie, the
    clearance from the edges (what is unique) and the radius;
  * the whole pipeline (prune, weighted layout, reinsert) over a few FP64
    iterations.
"""
import math
import os

import numpy as np
import pytest

import oracle
from gpu_common import pos_err, rel_l2, require_gpu
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _wheel(spokes, leaves):
    """Hub 0 joined to a ring 1..spokes, plus `leaves` degree-one vertices on
    the hub (ids after the ring)."""
    u = [0] * spokes + list(range(1, spokes + 1)) + [0] * leaves
    v = (list(range(1, spokes + 1)) + [1 + (i % spokes) for i in range(1, spokes + 1)] +
         list(range(spokes + 1, spokes + 1 + leaves)))
    return inputs.to_csr(spokes + 1 + leaves, u, v, name=f"wheel{spokes}+{leaves}")


def prune_suite():
    return [
        inputs.star_graph(300),
        inputs.path_graph(2),
        inputs.path_graph(300),
        inputs.to_csr(10, [0, 1, 5], [1, 2, 6], name="sparse10"),
        inputs.random_tree_plus_edges(2500, 600, seed=4),
        inputs.barabasi_albert(3000, 1, seed=7),          # a tree: most vertices are leaves
        inputs.barabasi_albert(3000, 2, seed=2),
        inputs.rmat(12, 4, 0.57, 0.19, 0.19, seed=3),
        inputs.grid_graph(16, 16),                        # nothing to prune
        _wheel(1000, 4),                                  # a row for the 256-thread sort
        _wheel(5000, 7),                                  # a long row: the 1024-thread sort
        _wheel(17000, 3),                                 # longer still: sorted in HBM
    ]


def _check_prune(G, g):
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    rp, ci = G.to_device_csr(g)
    P = G.prune(rp, ci)
    info = P.info()
    assert info["n_kept"] == pr.n
    assert info["nnz_kept"] == pr.col_idx.size
    assert info["n_pruned"] == g.n - pr.n
    assert info["n_with_leaves"] == int((pr.leaves > 0).sum())
    a, lv, ni = P.export()
    assert np.array_equal(a, pr.anchor) and np.array_equal(lv, pr.leaves)
    assert np.array_equal(ni, pr.new_id)
    return pr, P, (rp, ci)


def test_prune_bit_exact(G):
    for g in prune_suite():
        print(f"prune {g.name}", flush=True)
        pr, P, keep = _check_prune(G, g)
        csr, _ = P.graph()
        kh = G.KHop.from_csr(csr, 1)
        ptr, idx = kh.export()  # k = 1: the adjacency rows of the pruned graph
        assert np.array_equal(ptr, pr.row_ptr) and np.array_equal(idx, pr.col_idx), g.name
        kh.free()
        P.free()


def test_prune_empty_graph(G):
    import torch
    rp = torch.zeros(1, dtype=torch.int64, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    P = G.prune(rp, ci)
    assert P.info()["n_kept"] == 0 and P.info()["nnz_kept"] == 0


def test_prune_rejects_malformed(G):
    import torch
    rp = torch.tensor([0, 1, 1], dtype=torch.int64, device="cuda")  # 0 -> 1 without 1 -> 0
    ci = torch.tensor([1], dtype=torch.int32, device="cuda")
    with pytest.raises(G.GilaError) as e:
        G.prune(rp, ci)
    assert e.value.code == G.GILA_EINVAL


def _step_pair(G, kh, g_n, rp_np, ci_np, k, pos0, prec, mass):
    import torch
    dt = G.position_dtype(prec)
    pos = torch.from_numpy(pos0).to(dtype=dt, device="cuda").contiguous()
    F = torch.zeros((g_n, 2), dtype=torch.float64, device="cuda")
    D = torch.zeros((g_n, 2), dtype=torch.float64, device="cuda")
    params = G.LayoutParams(temperature=np.array([25.0]), ideal_length=40.0, precision=prec)
    st = G.step(kh, params, 0, pos, F, D)
    optr, oidx = oracle.khop(g_n, rp_np, ci_np, k)
    xo, Fo, Do, so = oracle.step(g_n, rp_np, ci_np, optr, oidx, 40.0, 25.0, pos0, mass=mass)
    return pos.double().cpu().numpy(), F.cpu().numpy(), st, xo, Fo, so


PATHS = {"segment": {}, "segment_tiny": {"GILA_SEG_BYTES": "2048"},
         "direct": {"GILA_PATH": "direct"}}


@pytest.fixture(params=list(PATHS))
def path_env(request):
    old = {k: os.environ.get(k) for k in ("GILA_PATH", "GILA_SEG_BYTES")}
    for k in old:
        os.environ.pop(k, None)
    os.environ.update(PATHS[request.param])
    yield request.param
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_kahan"])
def test_weighted_step_pruned_graphs(G, precision, path_env):
    """One step of each pruned graph with the pruning's weights (taken from
    the device handle), against the oracle's weighted step."""
    prec = G.PRECISIONS[precision]
    tol = 1e-12 if prec == G.FP64 else 1e-5
    for g in prune_suite():
        if g.name.startswith("wheel"):
            continue  # all pairs within two hops: covered by the reinsertion tests
        for k in (1, 2, 3):
            print(f"weighted {g.name} k={k} {precision} {path_env}", flush=True)
            pr, P, _ = _check_prune(G, g)
            csr, mass_addr = P.graph()
            kh = G.KHop.from_csr(csr, k)
            kh.set_mass(mass_addr)
            pos0 = inputs.uniform_positions(pr.n, seed=5, width=1200.0)
            if prec != G.FP64:
                pos0 = pos0.astype(np.float32).astype(np.float64)
            x_g, F_g, st, x_o, F_o, so = _step_pair(G, kh, pr.n, pr.row_ptr, pr.col_idx, k,
                                                     pos0, prec, pr.mass())
            assert rel_l2(F_g, F_o) <= tol, (g.name, k, rel_l2(F_g, F_o))
            if pr.n > 1:
                assert pos_err(x_g, x_o) <= tol, (g.name, k)
            assert st.coincident == so.coincident
            kh.free()
            P.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_arbitrary_weights_and_reset(G, precision, path_env):
    """Weights in [0, 5) (zeros included) on an unpruned graph; then
    set_mass(None) gives the unweighted handle's bits back."""
    import torch
    prec = G.PRECISIONS[precision]
    tol = 1e-12 if prec == G.FP64 else 1e-5
    g = inputs.barabasi_albert(4000, 3, seed=9)
    rp, ci = G.to_device_csr(g)
    rng = np.random.default_rng(1)
    w = rng.uniform(0.0, 5.0, g.n)
    w[rng.integers(0, g.n, 50)] = 0.0
    pos0 = inputs.uniform_positions(g.n, seed=8, width=1200.0)
    if prec != G.FP64:
        pos0 = pos0.astype(np.float32).astype(np.float64)
    kh = G.build_khop(rp, ci, 2)
    _, F_plain, _, _, _, _ = _step_pair(G, kh, g.n, g.row_ptr, g.col_idx, 2, pos0, prec, None)
    kh.set_mass(torch.from_numpy(w).cuda())
    x_g, F_g, _, x_o, F_o, _ = _step_pair(G, kh, g.n, g.row_ptr, g.col_idx, 2, pos0, prec, w)
    assert rel_l2(F_g, F_o) <= tol and pos_err(x_g, x_o) <= tol
    kh.set_mass(None)
    _, F_back, _, _, _, _ = _step_pair(G, kh, g.n, g.row_ptr, g.col_idx, 2, pos0, prec, None)
    assert np.array_equal(F_back, F_plain)
    # out-of-range weights are refused and the unit weights stay
    bad = torch.from_numpy(np.where(np.arange(g.n) == 7, -1.0, 1.0)).cuda()
    with pytest.raises(G.GilaError) as e:
        kh.set_mass(bad)
    assert e.value.code == G.GILA_EINVAL
    _, F_again, _, _, _, _ = _step_pair(G, kh, g.n, g.row_ptr, g.col_idx, 2, pos0, prec, None)
    assert np.array_equal(F_again, F_plain)


def test_weighted_run_graph_matches_steps(G):
    """gila_run (captured loop) with weights gives the same bits as steps."""
    import torch
    g = inputs.random_tree_plus_edges(3000, 900, seed=2)
    pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
    rp, ci = G.to_device_csr(g)
    P = G.prune(rp, ci)
    csr, m = P.graph()
    kh = G.KHop.from_csr(csr, 2)
    kh.set_mass(m)
    temps = G.paper_schedule(pr.n, 1.0, 40.0, 12)
    params = G.LayoutParams(temperature=temps, ideal_length=40.0, precision=G.FP32_KAHAN)
    pos0 = torch.from_numpy(inputs.uniform_positions(pr.n, 3, 1200.0)).float().cuda()
    a = pos0.clone()
    G.run(kh, params, a)
    b = pos0.clone()
    for h in range(12):
        G.step(kh, params, h, b)
    assert torch.equal(a, b)


def _clearance(rel_leaf, edge_vecs):
    th = np.arctan2(rel_leaf[:, 1], rel_leaf[:, 0])
    ea = np.arctan2(edge_vecs[:, 1], edge_vecs[:, 0])
    x = np.abs(th[:, None] - ea[None, :]) % (2 * math.pi)
    return float(np.minimum(x, 2 * math.pi - x).min())


def _gap_unique(pos_kept, pr, v, margin=1e-9):
    """True when the widest residue gap of kept vertex v beats the runner-up."""
    i = pr.new_id[v]
    nb = pr.col_idx[pr.row_ptr[i]:pr.row_ptr[i + 1]]
    if nb.size <= 1:
        return True
    L = pr.leaves[v]
    T = 2 * math.pi / L
    vec = pos_kept[nb] - pos_kept[i]
    r = np.sort(np.mod(np.mod(np.arctan2(vec[:, 1], vec[:, 0]), 2 * math.pi), T))
    gaps = np.diff(np.concatenate([r, [r[0] + T]]))
    top = np.sort(gaps)[-2:]
    return top[1] - top[0] > margin


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reinsert_parity(G, precision):
    import torch
    prec = G.PRECISIONS[precision]
    for g in prune_suite():
        print(f"reinsert {g.name} {precision}", flush=True)
        pr, P, _ = _check_prune(G, g)
        d = 40.0
        pk = inputs.uniform_positions(pr.n, seed=21, width=1200.0)
        if prec != G.FP64:
            pk = pk.astype(np.float32).astype(np.float64)
        dt = G.position_dtype(prec)
        pk_dev = torch.from_numpy(pk).to(dtype=dt, device="cuda").contiguous()
        out = torch.full((g.n, 2), float("nan"), dtype=dt, device="cuda")
        P.reinsert(d, prec, pk_dev, out)
        got = out.double().cpu().numpy()
        ref = oracle.reinsert(pr, d, pk)
        assert np.isfinite(got).all()
        kept = pr.new_id >= 0
        assert np.array_equal(got[kept], ref[kept])
        scale = max(1.0, float(np.abs(pk).max()) if pk.size else 1.0)
        atol = (1e-10 if prec == G.FP64 else 2.0 ** -21) * scale
        for v in np.flatnonzero(pr.leaves > 0):
            lv = np.flatnonzero(pr.anchor == v)
            i = pr.new_id[v]
            if _gap_unique(pk, pr, v):
                np.testing.assert_allclose(got[lv], ref[lv], rtol=0, atol=atol,
                                           err_msg=f"{g.name} vertex {v}")
            else:
                nb = pr.col_idx[pr.row_ptr[i]:pr.row_ptr[i + 1]]
                vec = pk[nb] - pk[i]
                assert abs(_clearance(got[lv] - pk[i], vec) -
                           _clearance(ref[lv] - pk[i], vec)) <= 1e-6
                np.testing.assert_allclose(np.hypot(*(got[lv] - pk[i]).T),
                                           np.hypot(*(ref[lv] - pk[i]).T), rtol=1e-6)
        P.free()


def test_reinsert_gather_roundtrip(G):
    import torch
    g = inputs.rmat(11, 4, 0.57, 0.19, 0.19, seed=8)
    pr, P, _ = _check_prune(G, g)
    full = torch.from_numpy(inputs.uniform_positions(g.n, 4, 1000.0)).cuda()
    kept = torch.empty((pr.n, 2), dtype=torch.float64, device="cuda")
    P.gather(G.FP64, full, kept)
    ids = np.flatnonzero(pr.new_id >= 0)
    assert torch.equal(kept.cpu(), full.cpu()[torch.from_numpy(ids)])


def test_pipeline_fp64(G):
    """gila_layout_pruned against the oracle's prune -> weighted layout ->
    reinsert, 6 FP64 iterations (short enough that rounding-order differences
    stay far below the gate)."""
    import torch
    for g in (inputs.random_tree_plus_edges(1500, 300, seed=6),
              inputs.barabasi_albert(2000, 1, seed=3)):
        print(f"pipeline {g.name}", flush=True)
        d, k, H = 30.0, 2, 6
        pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
        temps = G.paper_schedule(pr.n, 1.0, d, H)
        params = G.LayoutParams(temperature=temps, ideal_length=d, precision=G.FP64)
        x0 = inputs.uniform_positions(g.n, 2, 1200.0)
        pos = torch.from_numpy(x0).cuda()
        st = G.layout_pruned(*G.to_device_csr(g), k, params, pos)
        assert st.iterations_run == H
        optr, oidx = oracle.khop(pr.n, pr.row_ptr, pr.col_idx, k)
        xk = x0[pr.new_id >= 0]
        xk, run, _ = oracle.layout(pr.n, pr.row_ptr, pr.col_idx, optr, oidx, d, temps, xk,
                                   mass=pr.mass())
        ref = oracle.reinsert(pr, d, xk)
        assert pos_err(pos.cpu().numpy(), ref) <= 1e-9, pos_err(pos.cpu().numpy(), ref)
