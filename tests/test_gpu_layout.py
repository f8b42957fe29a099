"""GPU layout loop: device-resident runs against step-by-step runs (bitwise),
resume, HIP-graph vs eager launches, the halting rule, seeded placement, and
whole FP64 trajectories against the oracle."""
import os

import numpy as np
import pytest

import oracle
from gpu_common import oracle_rows, pos_err, require_gpu
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _t(G, x, prec):
    import torch
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).to(
        dtype=G.position_dtype(prec), device="cuda").contiguous()


def _np(t):
    return t.double().cpu().numpy()


def test_init_positions_match_generator(G):
    import torch
    for n, seed, w, h in [(1, 0, 1000.0, 1000.0), (1024, 0, 1000.0, 1000.0),
                          (100001, 12345, 1200.0, 700.0)]:
        ref = inputs.uniform_positions(n, seed, w, h)
        p64 = torch.empty((n, 2), dtype=torch.float64, device="cuda")
        G.init_positions(n, seed, w, h, G.FP64, p64)
        assert np.array_equal(_np(p64), ref)
        p32 = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        G.init_positions(n, seed, w, h, G.FP32, p32)
        assert np.array_equal(p32.cpu().numpy(), ref.astype(np.float32))


@pytest.mark.parametrize("path", ["segment", "direct"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_kahan"])
def test_run_equals_steps_and_resume(G, precision, path):
    prec = G.PRECISIONS[precision]
    if path == "direct":
        os.environ["GILA_PATH"] = "direct"
    try:
        _run_equals_steps_and_resume(G, prec)
    finally:
        os.environ.pop("GILA_PATH", None)


def _run_equals_steps_and_resume(G, prec):
    g = inputs.random_tree_plus_edges(3000, 1500, seed=21)
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, 3)
    H = 25
    params = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 48.0, H), ideal_length=48.0,
                            precision=prec)
    x0 = inputs.uniform_positions(g.n, seed=3, width=1200.0)
    a = _t(G, x0, prec)
    st = G.run(kh, params, a)
    assert st.iterations_run == H and st.stopped == 0
    b = _t(G, x0, prec)
    for h in range(H):
        G.step(kh, params, h, b)
    assert np.array_equal(_np(a), _np(b))
    c = _t(G, x0, prec)
    G.run(kh, params, c, 0, 9)
    G.run(kh, params, c, 9, H)
    assert np.array_equal(_np(a), _np(c))
    # eager launches (no HIP graph) give the same bits
    os.environ["GILA_NO_GRAPH"] = "1"
    try:
        e = _t(G, x0, prec)
        G.run(kh, params, e)
    finally:
        del os.environ["GILA_NO_GRAPH"]
    assert np.array_equal(_np(a), _np(e))
    # a second graph replay with fresh inputs repeats the first
    f = _t(G, x0, prec)
    G.run(kh, params, f)
    assert np.array_equal(_np(a), _np(f))


@pytest.mark.parametrize("path", ["segment", "direct"])
def test_long_run_in_chunks_equals_steps(G, path):
    """Runs of 100 or more iterations replay a captured chunk of iterations
    whose temperatures are read on the device: the result is bitwise that of
    single steps, of eager launches and of a run split at any iteration, the
    chunk is re-captured when the parameters change, and the history rows
    match the steps."""
    if path == "direct":
        os.environ["GILA_PATH"] = "direct"
    try:
        g = inputs.random_tree_plus_edges(1500, 700, seed=27)
        rp, ci = G.to_device_csr(g)
        kh = G.build_khop(rp, ci, 2)
        H = 137
        params = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 40.0, H),
                                ideal_length=40.0, precision=G.FP32_KAHAN)
        x0 = inputs.uniform_positions(g.n, seed=6, width=1000.0)
        kh.enable_history(H)
        a = _t(G, x0, G.FP32_KAHAN)
        st = G.run(kh, params, a)
        assert st.iterations_run == H and st.stopped == 0
        hist = kh.history()
        b = _t(G, x0, G.FP32_KAHAN)
        for h in range(H):
            sh = G.step(kh, params, h, b)
            assert tuple(hist[h]) == (sh.energy, sh.max_disp, float(sh.moved),
                                      float(sh.coincident)), h
        assert np.array_equal(_np(a), _np(b))
        c = _t(G, x0, G.FP32_KAHAN)
        G.run(kh, params, c, 0, 105)
        G.run(kh, params, c, 105, H)
        assert np.array_equal(_np(a), _np(c))
        os.environ["GILA_NO_GRAPH"] = "1"
        try:
            e = _t(G, x0, G.FP32_KAHAN)
            G.run(kh, params, e)
        finally:
            del os.environ["GILA_NO_GRAPH"]
        assert np.array_equal(_np(a), _np(e))
        # other parameters: the captured chunk must not be reused
        other = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 30.0, H),
                               ideal_length=30.0, precision=G.FP32_KAHAN)
        f = _t(G, x0, G.FP32_KAHAN)
        G.run(kh, other, f)
        os.environ["GILA_NO_GRAPH"] = "1"
        try:
            q = _t(G, x0, G.FP32_KAHAN)
            G.run(kh, other, q)
        finally:
            del os.environ["GILA_NO_GRAPH"]
        assert np.array_equal(_np(f), _np(q))
        assert not np.array_equal(_np(f), _np(a))
        kh.free()
    finally:
        os.environ.pop("GILA_PATH", None)


def test_grid_fp64_trajectory_matches_oracle(G):
    """Config-1 layout end to end (FP64, 100 iterations, device-resident loop).

    The layout dynamics are chaotic: in the oracle itself a one-ulp change of
    one coordinate grows to ~1e-2 of the extent by h = 100 (see
    test_oracle_trajectory_sensitivity), so whole trajectories agree only up
    to h ~ 40 (the GPU's differently ordered sums perturb every coordinate by
    ~1e-16 each step, so by h = 40 the trajectories differ by ~1e-8).  Parity
    is therefore checked (a) on the whole trajectory up to h = 40 and (b) step
    by step along the GPU's own trajectory to the end."""
    g = inputs.grid_graph(32, 32)
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, 2)
    temps = G.linear_schedule(100.0, 100)
    params = G.LayoutParams(temperature=temps, ideal_length=10.0, precision=G.FP64)
    import torch
    pos = torch.empty((g.n, 2), dtype=torch.float64, device="cuda")
    G.init_positions(g.n, 0, 1000.0, 1000.0, G.FP64, pos)
    x0 = _np(pos)
    optr, oidx = oracle_rows(g, 2)
    G.run(kh, params, pos, 0, 40)
    xo, run, _ = oracle.layout(g.n, g.row_ptr, g.col_idx, optr, oidx, 10.0, temps, x0, h_end=40)
    err40 = pos_err(_np(pos), xo)
    print(f"grid fp64 trajectory to h=40: e_x={err40:.3e}")
    assert err40 <= 1e-6
    worst = 0.0
    for h in range(40, 100):
        x_h = _np(pos)
        G.run(kh, params, pos, h, h + 1)
        x_o, _, _, _ = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 10.0, temps[h], x_h)
        worst = max(worst, pos_err(_np(pos), x_o))
    print(f"grid fp64 per-step along the device trajectory h=40..99: worst e_x={worst:.3e}")
    assert worst <= 1e-12


def test_halting_rule_matches_oracle(G):
    """The halting decision is an integer taken from the iteration's moves:
    the oracle, given the GPU's positions before the stopping iteration and
    the one before it, must take the same decisions."""
    g = inputs.watts_strogatz(600, 6, 0.1, seed=8)
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, 2)
    H = 400
    temps = G.paper_schedule(g.n, 1.0, 20.0, H)
    params = G.LayoutParams(temperature=temps, ideal_length=20.0, precision=G.FP64,
                            stop_fraction=0.15, stop_displacement=0.01)
    x0 = inputs.uniform_positions(g.n, seed=4, width=600.0)
    pos = _t(G, x0, G.FP64)
    st = G.run(kh, params, pos)
    print(f"halting after {st.iterations_run} iterations")
    assert st.stopped == 1 and 1 < st.iterations_run < H
    hs = st.iterations_run
    optr, oidx = oracle_rows(g, 2)
    nact = int((np.diff(g.row_ptr) > 0).sum())
    for h_last, expect_stop in ((hs - 2, False), (hs - 1, True)):
        p = _t(G, x0, G.FP64)
        G.run(kh, params, p, 0, h_last)
        _, _, _, so = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 20.0, temps[h_last],
                                  _np(p), stop_displacement=0.01)
        assert (so.moved < 0.15 * nact) == expect_stop, (h_last, so.moved)
    # the run that stopped left the positions of its last iteration
    q = _t(G, x0, G.FP64)
    G.run(kh, params.__class__(temperature=temps, ideal_length=20.0, precision=G.FP64), q, 0, hs)
    assert np.array_equal(_np(q), _np(pos))


def test_halting_on_symmetric_ring_matches_oracle_exactly(G):
    """A ring placed as a regular polygon moves every vertex alike, so the
    stop iteration is insensitive to rounding (a one-ulp perturbation changes
    the oracle's own positions by ~3e-3 of the extent by then, but not the
    iteration at which it stops): GPU and oracle stop at the same iteration."""
    n = 64
    g = inputs.cycle_graph(n)
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, 2)
    th = 2 * np.pi * np.arange(n) / n
    x0 = np.stack([200 * np.cos(th), 200 * np.sin(th)], axis=1)
    temps = 20.0 * 0.9 ** np.arange(300)
    params = G.LayoutParams(temperature=temps, ideal_length=10.0, precision=G.FP64,
                            stop_fraction=0.15, stop_displacement=0.01)
    pos = _t(G, x0, G.FP64)
    st = G.run(kh, params, pos)
    optr, oidx = oracle_rows(g, 2)
    xo, run, so = oracle.layout(g.n, g.row_ptr, g.col_idx, optr, oidx, 10.0, temps, x0,
                                stop_fraction=0.15, stop_displacement=0.01)
    print(f"ring halting after {st.iterations_run} (oracle {run})")
    assert st.stopped == 1 and st.iterations_run == run < 300


def test_zero_iterations_and_isolated_only(G):
    g = inputs.to_csr(50, [], [])
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, 2)
    x0 = inputs.uniform_positions(50, seed=1, width=10.0)
    pos = _t(G, x0, G.FP32)
    params = G.LayoutParams(temperature=np.ones(5), ideal_length=2.0, precision=G.FP32)
    st = G.run(kh, params, pos)
    assert np.array_equal(_np(pos), x0.astype(np.float32).astype(np.float64))
    assert st.iterations_run == 5
    g2 = inputs.grid_graph(4, 4)
    rp2, ci2 = G.to_device_csr(g2)
    kh2 = G.build_khop(rp2, ci2, 2)
    pos2 = _t(G, inputs.uniform_positions(16, seed=1, width=10.0), G.FP32)
    before = _np(pos2).copy()
    st = G.run(kh2, G.LayoutParams(temperature=np.ones(3), ideal_length=2.0, precision=G.FP32),
               pos2, 1, 1)
    assert st.iterations_run == 0 and np.array_equal(_np(pos2), before)


def test_layout_is_deterministic(G):
    g = inputs.rmat(13, 4, 0.57, 0.19, 0.19, seed=5)
    rp, ci = G.to_device_csr(g)
    params = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 48.0, 30), ideal_length=48.0,
                            precision=G.FP32_KAHAN)
    outs = []
    for _ in range(2):
        import torch
        pos = torch.empty((g.n, 2), dtype=torch.float32, device="cuda")
        G.init_positions(g.n, 7, 1200.0, 1200.0, G.FP32, pos)
        G.layout(rp, ci, 2, params, pos)
        outs.append(_np(pos))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("path", ["segment", "direct"])
def test_time_iterations_advances_like_run(G, path):
    """gila_time_iterations times graph replays (force kernel alone, then the
    iterations) and leaves the positions exactly where gila_run does; the
    force kernel's average does not exceed the iteration's."""
    if path == "direct":
        os.environ["GILA_PATH"] = "direct"
    try:
        g = inputs.random_tree_plus_edges(3000, 1500, seed=22)
        rp, ci = G.to_device_csr(g)
        kh = G.build_khop(rp, ci, 3)
        H = 12
        params = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 48.0, H),
                                ideal_length=48.0, precision=G.FP32_KAHAN)
        x0 = inputs.uniform_positions(g.n, seed=4, width=1200.0)
        a = _t(G, x0, G.FP32_KAHAN)
        G.run(kh, params, a, 0, 4)
        G.run(kh, params, a, 4, H)
        b = _t(G, x0, G.FP32_KAHAN)
        G.run(kh, params, b, 0, 4)
        force_ms, rest_ms, in_graph = G.time_iterations(kh, params, b, 4, H - 4, with_mode=True)
        assert np.array_equal(_np(a), _np(b))
        assert in_graph
        assert force_ms > 0.0 and rest_ms >= 0.0, (force_ms, rest_ms)
        if path == "direct":
            assert rest_ms == 0.0
        with pytest.raises(G.GilaError):
            G.time_iterations(kh, params, b, 4, H)     # beyond the schedule
        kh.free()
    finally:
        os.environ.pop("GILA_PATH", None)


@pytest.mark.parametrize("path", ["segment", "direct"])
def test_history_rows_equal_step_statistics(G, path):
    """Per-iteration history: each row of a run equals the statistics the same
    iteration reports when taken alone (bitwise), rows past the schedule and
    after the halting rule stopped the run stay NaN, and the table's bounds
    are checked."""
    if path == "direct":
        os.environ["GILA_PATH"] = "direct"
    try:
        g = inputs.random_tree_plus_edges(2000, 1000, seed=23)
        rp, ci = G.to_device_csr(g)
        kh = G.build_khop(rp, ci, 2)
        H = 15
        params = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 48.0, H),
                                ideal_length=48.0, precision=G.FP32_KAHAN)
        x0 = inputs.uniform_positions(g.n, seed=5, width=1200.0)
        kh.enable_history(H + 5)
        a = _t(G, x0, G.FP32_KAHAN)
        st = G.run(kh, params, a)
        hist = kh.history()
        assert hist.shape == (H + 5, 4)
        assert np.isnan(hist[H:]).all() and np.isfinite(hist[:H]).all()
        assert tuple(hist[H - 1]) == (st.energy, st.max_disp, float(st.moved), float(st.coincident))
        b = _t(G, x0, G.FP32_KAHAN)
        for h in range(H):
            sh = G.step(kh, params, h, b)
            assert tuple(hist[h]) == (sh.energy, sh.max_disp, float(sh.moved),
                                      float(sh.coincident)), h
        # the halting rule: rows after the last iteration run stay NaN
        long = G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 48.0, 400), ideal_length=48.0,
                              precision=G.FP32_KAHAN, stop_fraction=0.15)
        kh.enable_history(400)
        c = _t(G, x0, G.FP32_KAHAN)
        st = G.run(kh, long, c)
        r = st.iterations_run
        assert st.stopped == 1 and r < 400
        hist = kh.history()
        assert np.isfinite(hist[:r]).all() and np.isnan(hist[r:]).all()
        assert hist[r - 1, 2] < 0.15 * int((np.diff(g.row_ptr) > 0).sum())
        with pytest.raises(G.GilaError):
            kh.history(395, 10)
        kh.enable_history(0)
        kh.free()
    finally:
        os.environ.pop("GILA_PATH", None)
