"""GPU parity of one layout iteration (forces, capped move) against the FP64
oracle, from identical positions.

Gates (relative, as stated for the layout): the force field
e_F = ||F_gpu - F_orc||_2 / ||F_orc||_2 <= 1e-5 and the positions
e_x = max_v |x_gpu - x_orc| / extent <= 1e-5.  FP64 runs are held to 1e-12.
The displacement error e_D is reported, not gated: near equilibrium a capped
move's direction is ill-conditioned, so FP32 per-term rounding shows up in it
whatever the summation method.
"""
import os

import numpy as np
import pytest

import oracle
from gpu_common import (oracle_rows, per_vertex_force_err, pos_err, rel_l2, require_gpu,
                        small_graph_suite)
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _dev(G, g):
    return G.to_device_csr(g)


def _gpu_step(G, kh, params, h, pos_np):
    import torch
    dt = G.position_dtype(params.precision)
    pos = torch.from_numpy(pos_np.astype(np.float64)).to(dtype=dt, device="cuda").contiguous()
    n = pos_np.shape[0]
    F = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    D = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    st = G.step(kh, params, h, pos, F, D)
    return (pos.double().cpu().numpy(), F.cpu().numpy(), D.cpu().numpy(), st)


PATHS = {
    "segment": {},                                   # LDS segments of 64 KB
    "segment_tiny": {"GILA_SEG_BYTES": "2048"},      # 2 KB segments: many segments per graph
    # every slice of 64 or more ids as a slot bitmap evaluated densely (FP32)
    "segment_dense": {"GILA_DENSE_MIN": "1"},
    "direct": {"GILA_PATH": "direct"},               # direct global gathers
}


@pytest.fixture(params=list(PATHS))
def path_env(request):
    old = {k: os.environ.get(k) for k in ("GILA_PATH", "GILA_SEG_BYTES", "GILA_DENSE_MIN")}
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
def test_single_step_small_suite(G, precision, path_env):
    prec = G.PRECISIONS[precision]
    for g in small_graph_suite():
        for k in (1, 2, 3):
            print(f"step {g.name} k={k} {precision} {path_env}", flush=True)
            rp, ci = _dev(G, g)
            kh = G.build_khop(rp, ci, k)
            pos0 = inputs.uniform_positions(g.n, seed=11, width=1200.0)
            if prec != G.FP64:
                pos0 = pos0.astype(np.float32).astype(np.float64)
            params = G.LayoutParams(temperature=np.array([30.0, 5.0]), ideal_length=48.0,
                                    precision=prec)
            x_g, F_g, D_g, st_g = _gpu_step(G, kh, params, 0, pos0)
            optr, oidx = oracle_rows(g, k)
            x_o, F_o, D_o, st_o = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 48.0, 30.0,
                                              pos0)
            tol = 1e-12 if prec == G.FP64 else 1e-5
            assert rel_l2(F_g, F_o) <= tol, (g.name, k, rel_l2(F_g, F_o))
            S = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, optr, oidx, 48.0, pos0)
            pv = per_vertex_force_err(F_g, F_o, S)
            assert pv <= tol, (g.name, k, pv)
            if g.n > 1:
                assert pos_err(x_g, x_o) <= tol, (g.name, k)
            assert st_g.iterations_run == 1
            assert st_g.coincident == st_o.coincident
            np.testing.assert_allclose(st_g.energy, st_o.energy, rtol=tol * 10)
            np.testing.assert_allclose(st_g.max_disp, st_o.max_disp, rtol=tol * 10)
            if prec == G.FP64:
                assert st_g.moved == st_o.moved
            kh.free()


def test_grid_fp64_every_step(G):
    """Config-1 shape: 32x32 grid, k = 2, d = 10, [0,1000)^2 from seed 0,
    linear cap from 100 over 100 iterations, FP64: every step from the same
    positions as the oracle's."""
    g = inputs.grid_graph(32, 32)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, 2)
    optr, oidx = oracle_rows(g, 2)
    temps = G.linear_schedule(100.0, 100)
    params = G.LayoutParams(temperature=temps, ideal_length=10.0, precision=G.FP64)
    x = inputs.uniform_positions(g.n, seed=0, width=1000.0)
    worst = (0.0, 0.0, 0.0)
    for h in range(100):
        x_g, F_g, D_g, _ = _gpu_step(G, kh, params, h, x)
        x_o, F_o, D_o, _ = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 10.0, temps[h], x)
        eF, ex, eD = rel_l2(F_g, F_o), pos_err(x_g, x_o), rel_l2(D_g, D_o)
        worst = tuple(max(a, b) for a, b in zip(worst, (eF, ex, eD)))
        x = x_o
    print(f"grid fp64 worst e_F={worst[0]:.3e} e_x={worst[1]:.3e} e_D={worst[2]:.3e}")
    assert worst[0] <= 1e-12 and worst[1] <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp32_kahan"])
def test_trajectory_sampled_steps_fp32(G, precision):
    """A 120-iteration layout of a BA graph (k = 3) driven by the GPU; at
    sampled steps the oracle recomputes the step from the GPU's positions."""
    prec = G.PRECISIONS[precision]
    g = inputs.barabasi_albert(6000, 3, seed=12)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, 3)
    optr, oidx = oracle_rows(g, 3)
    H = 120
    d = inputs.PAPER_IDEAL_LENGTH
    temps = G.paper_schedule(g.n, 1.0, d, H)
    params = G.LayoutParams(temperature=temps, ideal_length=d, precision=prec)
    x = inputs.uniform_positions(g.n, seed=0, width=1200.0).astype(np.float32).astype(np.float64)
    checked = {0, H // 10, H // 4, H // 2, 3 * H // 4, H - 1}
    for h in range(H):
        x_g, F_g, D_g, _ = _gpu_step(G, kh, params, h, x)
        if h in checked:
            x_o, F_o, D_o, _ = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, d, temps[h], x)
            eF, ex, eD = rel_l2(F_g, F_o), pos_err(x_g, x_o), rel_l2(D_g, D_o)
            print(f"{precision} h={h} e_F={eF:.2e} e_x={ex:.2e} e_D={eD:.2e}", flush=True)
            assert eF <= 1e-5 and ex <= 1e-5, (h, eF, ex)
        x = x_g


@pytest.mark.parametrize("which", ["rmat18_k2", "ba100k_k3"])
def test_full_size_step(G, which, path_env):
    """Full benchmark graphs, FP32 + Kahan, first and a later step: whole
    force field against the oracle."""
    if which == "rmat18_k2":
        g, k, frame = inputs.rmat(18, 4, 0.57, 0.19, 0.19, seed=3), 2, 1200.0
    else:
        g, k, frame = inputs.barabasi_albert(100000, 3, seed=2), 3, 1e4
    if path_env == "segment_tiny":
        pytest.skip("tiny segments are exercised on the small suite")
    print(f"full-size step {which} {path_env}", flush=True)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, k)
    optr, oidx = oracle_rows(g, k)
    d = inputs.PAPER_IDEAL_LENGTH
    temps = G.paper_schedule((np.diff(g.row_ptr) > 0).sum(), 1.0, d, 40)
    params = G.LayoutParams(temperature=temps, ideal_length=d, precision=G.FP32_KAHAN)
    x = inputs.uniform_positions(g.n, seed=0, width=frame).astype(np.float32).astype(np.float64)
    for h in range(3):
        x_g, F_g, D_g, st = _gpu_step(G, kh, params, h, x)
        x_o, F_o, D_o, so = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, d, temps[h], x)
        S = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, optr, oidx, d, x)
        eF, ex, eD = rel_l2(F_g, F_o), pos_err(x_g, x_o), rel_l2(D_g, D_o)
        pv = per_vertex_force_err(F_g, F_o, S)
        print(f"{which} {path_env} h={h} e_F={eF:.2e} e_x={ex:.2e} e_D={eD:.2e} "
              f"max|dF_v|/S_v={pv:.2e}", flush=True)
        assert eF <= 1e-5 and ex <= 1e-5 and pv <= 1e-5
        assert st.coincident == so.coincident
        x = x_g
    del oidx


def test_cap_extremes(G):
    g = inputs.barabasi_albert(500, 2, seed=3)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, 2)
    x = inputs.uniform_positions(g.n, seed=1, width=300.0)
    # t = 0 moves nothing
    p0 = G.LayoutParams(temperature=np.array([0.0]), ideal_length=20.0, precision=G.FP64)
    x_g, F_g, D_g, st = _gpu_step(G, kh, p0, 0, x)
    assert np.array_equal(x_g, x) and st.moved == 0 and st.max_disp == 0.0
    # a huge cap gives Delta = F exactly
    p1 = G.LayoutParams(temperature=np.array([1e30]), ideal_length=20.0, precision=G.FP64)
    x_g, F_g, D_g, st = _gpu_step(G, kh, p1, 0, x)
    assert np.array_equal(D_g, F_g)


def test_coincident_vertices(G):
    g = inputs.path_graph(3)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, 2)
    x = np.array([[0.0, 0.0], [0.0, 0.0], [4.0, 0.0]])
    p = G.LayoutParams(temperature=np.array([1.0]), ideal_length=2.0, precision=G.FP32_KAHAN)
    x_g, F_g, D_g, st = _gpu_step(G, kh, p, 0, x)
    assert st.coincident == 2
    assert np.all(np.isfinite(F_g)) and np.all(np.isfinite(x_g))
    np.testing.assert_allclose(F_g[0], [-1.0, 0.0], rtol=1e-6)


@pytest.mark.parametrize("k", [1, 2])
def test_dense_slice_coincident_and_forces(G, k, monkeypatch):
    """Rows of 100 ids stored as slot bitmaps (GILA_DENSE_MIN=1 makes every
    slice of 64 or more ids dense): forces and move match the oracle, and the
    coincident pairs (three leaves placed on the hub) are counted exactly."""
    monkeypatch.setenv("GILA_DENSE_MIN", "1")
    g = inputs.star_graph(100)
    rp, ci = _dev(G, g)
    kh = G.build_khop(rp, ci, k)
    x = inputs.uniform_positions(g.n, seed=4, width=300.0).astype(np.float32).astype(np.float64)
    for leaf in (5, 17, 60):
        x[leaf] = x[0]
    params = G.LayoutParams(temperature=np.array([10.0]), ideal_length=20.0,
                            precision=G.FP32_KAHAN)
    x_g, F_g, D_g, st = _gpu_step(G, kh, params, 0, x)
    optr, oidx = oracle_rows(g, k)
    x_o, F_o, D_o, so = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 20.0, 10.0, x)
    assert so.coincident > 0 and st.coincident == so.coincident
    S = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, optr, oidx, 20.0, x)
    assert rel_l2(F_g, F_o) <= 1e-5
    assert per_vertex_force_err(F_g, F_o, S) <= 1e-5
    assert pos_err(x_g, x_o) <= 1e-5
    kh.free()
