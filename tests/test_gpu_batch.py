"""GPU parity of the batched form: many graphs of mixed sizes, families and k
in one persistent launch, each graph's iterations run in LDS.

Checks: one FP64 iteration with an unbounded cap returns x + F exactly, so
the batch's forces are compared with the oracle's at 1e-12; FP32 + Kahan
iterations stepped along each graph's own trajectory against the oracle at
the 1e-5 gates; a graph alone and inside a batch give the same bits; the
halting rule per graph; malformed inputs are rejected."""
import numpy as np
import pytest

import oracle
from gpu_common import oracle_rows, pos_err, rel_l2, require_gpu
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _mixed_graphs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    sizes = inputs.log_uniform_sizes(count, 20, 3000, seed)
    for i, n in enumerate(sizes.tolist()):
        fam = i % 4
        if fam == 0:
            g = inputs.random_tree_plus_edges(n, n // 2, seed=seed * 100 + i)
        elif fam == 1:
            g = inputs.watts_strogatz(max(n, 8), 6, 0.1, seed=seed * 100 + i)
        elif fam == 2:
            g = inputs.barabasi_albert(max(n, 5), 2, seed=seed * 100 + i)
        else:
            side = max(2, int(np.sqrt(n)))
            g = inputs.grid_graph(side, side)
        out.append((g, int(rng.integers(1, 4))))
    return out


def _t(G, x, prec):
    import torch
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).to(
        dtype=G.position_dtype(prec), device="cuda").contiguous()


@pytest.mark.parametrize("bfs", ["graph", "source"])
def test_batch_khop_lists_bit_exact(G, bfs, monkeypatch):
    """Every graph's k-hop lists equal the oracle's BFS, on the per-graph LDS
    path and on the per-source path (GILA_BATCH_BFS=source)."""
    if bfs == "source":
        monkeypatch.setenv("GILA_BATCH_BFS", "source")
    gs = _mixed_graphs(60, 7)
    gs.append((inputs.path_graph(2), 5))        # k beyond the diameter
    gs.append((inputs.complete_graph(40), 2))   # dense rows
    gs.append((inputs.Graph(n=3, row_ptr=np.zeros(4, np.int64), col_idx=np.zeros(0, np.int32)), 2))
    dev = [G.to_device_csr(g) for g, _ in gs]
    b = G.Batch(dev, [k for _, k in gs])
    for i, (g, k) in enumerate(gs):
        ptr, idx = b.export(i, g.n)
        optr, oidx = oracle_rows(g, k)
        assert np.array_equal(ptr, optr), (i, g.name, k)
        assert np.array_equal(idx, oidx), (i, g.name, k)
    b.free()


def test_batch_khop_half_size_workgroups_bit_exact(G):
    """A batch whose largest graph leaves no room in LDS for the bitmaps of 16
    wavefronts beside its CSR (11,000 vertices, ~33,000 adjacency entries:
    ~176 KB) runs the one-pass build in 512-thread workgroups (~143 KB); its
    lists, and those of the small graphs beside it, equal the oracle's."""
    gs = [(inputs.random_tree_plus_edges(11000, 5500, seed=81), 2),
          (inputs.barabasi_albert(400, 2, seed=82), 3),
          (inputs.random_tree_plus_edges(60, 30, seed=83), 4)]
    nmax = max(g.n for g, _ in gs)
    nnzmax = max(int(g.row_ptr[-1]) for g, _ in gs)

    def bfs_lds(waves):  # the build's LDS budget of the one-pass BFS
        return 4 * (nmax + 1) + 2 * ((nnzmax + 1) & ~1) + 4 * ((nmax + 31) // 32) * 3 * waves

    assert bfs_lds(16) + 1024 > 160 * 1024 >= bfs_lds(8) + 1024
    b = G.Batch([G.to_device_csr(g) for g, _ in gs], [k for _, k in gs])
    for i, (g, k) in enumerate(gs):
        ptr, idx = b.export(i, g.n)
        optr, oidx = oracle_rows(g, k)
        assert np.array_equal(ptr, optr), (i, g.name, k)
        assert np.array_equal(idx, oidx), (i, g.name, k)
    b.free()


def test_concatenated_marshalling_same_bits(G):
    """Batch.concatenated + BatchParams + (positions, offsets) give the same
    bits as the per-graph list form."""
    import torch
    gs = _mixed_graphs(30, 9)
    ks = [k for _, k in gs]
    H = 25
    temps = [G.paper_schedule(max(g.n, 1), 1.0, 40.0, H) for g, _ in gs]
    x0 = [inputs.uniform_positions(g.n, seed=i, width=800.0) for i, (g, _) in enumerate(gs)]
    # list form
    dev = [G.to_device_csr(g) for g, _ in gs]
    pos_list = [_t(G, x, G.FP32) for x in x0]
    params = [G.LayoutParams(temperature=t, ideal_length=40.0, precision=G.FP32) for t in temps]
    b1 = G.Batch(dev, ks)
    st1 = b1.run(params, pos_list)
    # concatenated form
    rp_all = torch.from_numpy(np.concatenate([g.row_ptr for g, _ in gs])).cuda()
    ci_all = torch.from_numpy(np.concatenate([g.col_idx for g, _ in gs])).cuda()
    n = np.array([g.n for g, _ in gs])
    nnz = np.array([g.nnz for g, _ in gs])
    voff = np.concatenate([[0], np.cumsum(n)[:-1]])
    pos_all = _t(G, np.concatenate(x0), G.FP32)
    b2 = G.Batch.concatenated(rp_all, ci_all, n, nnz, ks)
    st2 = b2.run(G.BatchParams(temps, 40.0, G.FP32), (pos_all, voff))
    for i in range(len(gs)):
        assert np.array_equal(pos_list[i].cpu().numpy(),
                              pos_all[voff[i]:voff[i] + n[i]].cpu().numpy()), i
        assert st1[i].iterations_run == st2[i].iterations_run == H
        assert st1[i].energy == st2[i].energy
    b1.free()
    b2.free()


def test_batch_fp64_forces_exact(G):
    gs = _mixed_graphs(40, 1)
    dev = [G.to_device_csr(g) for g, _ in gs]
    b = G.Batch(dev, [k for _, k in gs])
    x0 = [inputs.uniform_positions(g.n, seed=i, width=500.0) for i, (g, _) in enumerate(gs)]
    pos = [_t(G, x, G.FP64) for x in x0]
    params = [G.LayoutParams(temperature=np.array([1e300]), ideal_length=30.0, precision=G.FP64)
              for _ in gs]
    st = b.run(params, pos)
    worst = 0.0
    for i, (g, k) in enumerate(gs):
        optr, oidx = oracle_rows(g, k)
        F, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, optr, oidx, 30.0, x0[i])
        Fg = pos[i].cpu().numpy() - x0[i]
        e = rel_l2(Fg, F)
        worst = max(worst, e)
        assert e <= 1e-10, (i, g.name, k, e)
        assert st[i].iterations_run == 1
    print(f"batch fp64 worst force error {worst:.3e}")


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32"])
def test_batch_steps_along_trajectory(G, precision):
    prec = G.PRECISIONS[precision]
    gs = _mixed_graphs(24, 2)
    dev = [G.to_device_csr(g) for g, _ in gs]
    b = G.Batch(dev, [k for _, k in gs])
    H = 30
    temps = [G.paper_schedule(g.n, 1.0, 40.0, H) for g, _ in gs]
    xs = [inputs.uniform_positions(g.n, seed=i, width=800.0).astype(np.float32).astype(np.float64)
          for i, (g, _) in enumerate(gs)]
    rows = [oracle_rows(g, k) for g, k in gs]
    worst = 0.0
    for h in range(H):
        pos = [_t(G, x, prec) for x in xs]
        params = [G.LayoutParams(temperature=temps[i][h:h + 1], ideal_length=40.0, precision=prec)
                  for i in range(len(gs))]
        b.run(params, pos)
        for i, (g, k) in enumerate(gs):
            xn = pos[i].double().cpu().numpy()
            if h % 7 == 0 or h == H - 1:
                xo, _, _, _ = oracle.step(g.n, g.row_ptr, g.col_idx, rows[i][0], rows[i][1], 40.0,
                                          temps[i][h], xs[i])
                e = pos_err(xn, xo) if g.n > 1 else 0.0
                worst = max(worst, e)
                assert e <= 1e-5, (h, i, g.name, e)
            xs[i] = xn
    print(f"batch {precision} worst per-step position error {worst:.3e}")


def test_alone_equals_mixed_bitwise(G):
    gs = _mixed_graphs(32, 3)
    dev = [G.to_device_csr(g) for g, _ in gs]
    H = 40
    params = [G.LayoutParams(temperature=G.paper_schedule(g.n, 1.0, 40.0, H), ideal_length=40.0,
                             precision=G.FP32_KAHAN) for g, _ in gs]
    x0 = [inputs.uniform_positions(g.n, seed=i, width=800.0) for i, (g, _) in enumerate(gs)]
    pos = [_t(G, x, G.FP32_KAHAN) for x in x0]
    G.Batch(dev, [k for _, k in gs]).run(params, pos)
    for i in (0, 5, 17, 31):
        alone = [_t(G, x0[i], G.FP32_KAHAN)]
        G.Batch([dev[i]], [gs[i][1]]).run([params[i]], alone)
        assert np.array_equal(alone[0].cpu().numpy(), pos[i].cpu().numpy()), i
    # and a second mix in another order
    perm = list(reversed(range(len(gs))))
    pos2 = [_t(G, x0[i], G.FP32_KAHAN) for i in perm]
    G.Batch([dev[i] for i in perm], [gs[i][1] for i in perm]).run([params[i] for i in perm], pos2)
    for j, i in enumerate(perm):
        assert np.array_equal(pos2[j].cpu().numpy(), pos[i].cpu().numpy()), i


def test_batch_halting_and_layout_batch(G):
    n = 64
    ring = inputs.cycle_graph(n)
    th = 2 * np.pi * np.arange(n) / n
    xr = np.stack([200 * np.cos(th), 200 * np.sin(th)], axis=1)
    temps = 20.0 * 0.9 ** np.arange(300)
    optr, oidx = oracle_rows(ring, 2)
    _, run, _ = oracle.layout(ring.n, ring.row_ptr, ring.col_idx, optr, oidx, 10.0, temps, xr,
                              stop_fraction=0.15, stop_displacement=0.01)
    other = inputs.random_tree_plus_edges(500, 250, seed=9)
    dev = [G.to_device_csr(ring), G.to_device_csr(other)]
    pos = [_t(G, xr, G.FP64), _t(G, inputs.uniform_positions(500, 1, 300.0), G.FP64)]
    params = [G.LayoutParams(temperature=temps, ideal_length=10.0, precision=G.FP64,
                             stop_fraction=0.15, stop_displacement=0.01),
              G.LayoutParams(temperature=temps[:50], ideal_length=10.0, precision=G.FP64)]
    st = G.layout_batch(dev, [2, 3], params, pos)
    assert st[0].stopped == 1 and st[0].iterations_run == run < 300
    assert st[1].stopped == 0 and st[1].iterations_run == 50


def test_batch_edge_cases(G):
    import torch
    # empty batch
    assert G.Batch([], []).run([], []) == []
    # a batch holding an isolated-only graph and a one-edge graph
    iso = inputs.to_csr(5, [], [])
    one = inputs.path_graph(2)
    dev = [G.to_device_csr(iso), G.to_device_csr(one)]
    x = [inputs.uniform_positions(5, 1, 10.0), np.array([[0.0, 0.0], [1.0, 0.0]])]
    pos = [_t(G, xi, G.FP64) for xi in x]
    p = G.LayoutParams(temperature=np.ones(3), ideal_length=4.0, precision=G.FP64)
    st = G.Batch(dev, [2, 1]).run([p, p], pos)
    assert np.array_equal(pos[0].cpu().numpy(), x[0])
    assert pos[1].cpu().numpy()[1, 0] > 1.0          # the pair repels apart (d = 4)
    assert st[0].iterations_run == 3
    # malformed graphs
    bad = (torch.tensor([0, 1, 1], dtype=torch.int64, device="cuda"),
           torch.tensor([1], dtype=torch.int32, device="cuda"))
    with pytest.raises(G.GilaError) as e:
        G.Batch([dev[1], bad], [1, 1])
    assert e.value.code == G.GILA_EINVAL
    with pytest.raises(G.GilaError):
        G.Batch([dev[1]], [0])
    # mixed precisions are refused
    b = G.Batch(dev, [2, 1])
    with pytest.raises(G.GilaError):
        b.run([p, G.LayoutParams(temperature=np.ones(3), ideal_length=4.0, precision=G.FP32)],
              pos)


def test_plan_is_fixed_at_build_and_reproducible(G):
    """Each graph's lanes per vertex (its summation order, hence its bits) is
    fixed at build from its mean row length -- the same for the same graph in
    any batch or process -- and a tuned plan read back and set on a fresh
    handle reproduces the tuned run's bits without tuning again."""
    import torch
    gs = _mixed_graphs(48, 13)
    dev = [G.to_device_csr(g) for g, _ in gs]
    ks = [k for _, k in gs]
    H = 6
    temps = [G.paper_schedule(max(g.n, 1), 1.0, 40.0, H) for g, _ in gs]
    params = [G.LayoutParams(temperature=t, ideal_length=40.0, precision=G.FP32_KAHAN)
              for t in temps]
    x0 = [inputs.uniform_positions(g.n, seed=i, width=900.0) for i, (g, _) in enumerate(gs)]

    def run(b):
        pos = [_t(G, x, G.FP32_KAHAN) for x in x0]
        b.run(params, pos)
        return [p.cpu() for p in pos]

    b1 = G.Batch(dev, ks)
    lanes1, cls1 = b1.plan()
    # the rule: one lane per vertex up to a class upper mean length of 128,
    # then about 128 entries per lane, and for small graphs at least the
    # lanes that fill 512 threads
    for (g, _), lanes, c in zip(gs, lanes1, cls1):
        want = 1
        while want < 64 and want * 128 < (4 << int(c)):
            want *= 2
        fill = 1
        while fill < 64 and g.n * fill * 2 <= 512:
            fill *= 2
        assert lanes == max(want, fill), (g.n, lanes, want, fill)
    a = run(b1)
    # a graph's plan does not depend on its batch: every 3rd graph alone
    sub = list(range(0, len(gs), 3))
    b2 = G.Batch([dev[i] for i in sub], [ks[i] for i in sub])
    assert np.array_equal(b2.plan()[0], lanes1[sub])
    b2.free()
    # tuned plan, read back, set on a new handle: the same bits
    table = b1.tune(G.FP32_KAHAN)
    assert table.shape == (8,) and all(v == 0 or v in (1, 2, 4, 8, 16, 32, 64) for v in table)
    lanes_t, _ = b1.plan()
    for (g, _), l, c in zip(gs, lanes_t, cls1):
        fill = 1
        while fill < 64 and g.n * fill * 2 <= 512:
            fill *= 2
        assert l == max(table[c], fill)
    tuned = run(b1)
    b3 = G.Batch(dev, ks)
    assert np.array_equal(b3.plan()[0], lanes1)        # a fresh handle starts from the rule
    b3.set_plan(lanes_t)
    again = run(b3)
    for x, y in zip(tuned, again):
        assert torch.equal(x, y)
    # and the rule's plan set back gives the first run's bits
    b3.set_plan(lanes1)
    for x, y in zip(a, run(b3)):
        assert torch.equal(x, y)
    with pytest.raises(G.GilaError) as e:
        b3.set_plan(np.full(len(gs), 3))
    assert e.value.code == G.GILA_EINVAL
    with pytest.raises(G.GilaError):
        b3.set_plan(np.full(len(gs), 128))
    b1.free()
    b3.free()


def test_wave_slices_forces_stats_and_large_graph(G):
    """Graphs planned at one lane per vertex run from wave slices: FP64 forces
    (one iteration, unbounded cap) and every statistic against the oracle,
    with a coincident pair inside a row; and, in FP32, a 9,000-vertex graph
    (beyond the sorted-order limit of 8,192, so its slices keep the identity
    order) stepped against the oracle at the 1e-5 gate."""
    gs = [(inputs.random_tree_plus_edges(300, 150, seed=31), 3),
          (inputs.watts_strogatz(1000, 6, 0.1, seed=32), 2),
          (inputs.barabasi_albert(2500, 2, seed=33), 2)]
    dev = [G.to_device_csr(g) for g, _ in gs]
    b = G.Batch(dev, [k for _, k in gs])
    lanes, _ = b.plan()
    assert (lanes == 1).all(), lanes
    x0 = [inputs.uniform_positions(g.n, seed=40 + i, width=700.0) for i, (g, _) in enumerate(gs)]
    g0 = gs[0][0]
    u = int(g0.col_idx[g0.row_ptr[5]])
    x0[0][u] = x0[0][5]                        # a coincident pair, one hop apart
    pos = [_t(G, x, G.FP64) for x in x0]
    params = [G.LayoutParams(temperature=np.array([1e300]), ideal_length=30.0, precision=G.FP64)
              for _ in gs]
    st = b.run(params, pos)
    for i, (g, k) in enumerate(gs):
        optr, oidx = oracle_rows(g, k)
        xo, F, D, ost = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 30.0, 1e300, x0[i])
        Fg = pos[i].cpu().numpy() - x0[i]
        assert rel_l2(Fg, F) <= 1e-10, (i, rel_l2(Fg, F))
        assert st[i].coincident == ost.coincident, (i, st[i].coincident, ost.coincident)
        assert st[i].moved == ost.moved, (i, st[i].moved, ost.moved)
        assert abs(st[i].energy - ost.energy) <= 1e-10 * ost.energy, (i, st[i].energy, ost.energy)
        assert abs(st[i].max_disp - ost.max_disp) <= 1e-10 * ost.max_disp, i
    assert st[0].coincident > 0
    b.free()

    big = inputs.random_tree_plus_edges(9000, 4500, seed=34)
    small = inputs.random_tree_plus_edges(700, 350, seed=35)
    gs = [(big, 2), (small, 3)]
    b = G.Batch([G.to_device_csr(g) for g, _ in gs], [k for _, k in gs])
    assert (b.plan()[0] == 1).all()
    rows = [oracle_rows(g, k) for g, k in gs]
    xs = [inputs.uniform_positions(g.n, seed=50 + i, width=1200.0).astype(np.float32)
          .astype(np.float64) for i, (g, _) in enumerate(gs)]
    H = 4
    temps = [G.paper_schedule(g.n, 1.0, 40.0, H) for g, _ in gs]
    for h in range(H):
        pos = [_t(G, x, G.FP32) for x in xs]
        params = [G.LayoutParams(temperature=temps[i][h:h + 1], ideal_length=40.0,
                                 precision=G.FP32) for i in range(len(gs))]
        st = b.run(params, pos)
        for i, (g, k) in enumerate(gs):
            xo, _, _, ost = oracle.step(g.n, g.row_ptr, g.col_idx, rows[i][0], rows[i][1], 40.0,
                                        temps[i][h], xs[i])
            xn = pos[i].double().cpu().numpy()
            assert pos_err(xn, xo) <= 1e-5, (h, i, pos_err(xn, xo))
            assert abs(st[i].energy - ost.energy) <= 1e-4 * ost.energy, (h, i)
            xs[i] = xn
    b.free()
