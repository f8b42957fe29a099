"""Both internal vertex orders give the oracle's forces.

gila_build_khop relabels vertices either by decreasing |N_v(k)| (degree
order) or, when most edges are short in the caller's numbering, keeping the
caller's order with long rows first (caller order); GILA_ORDER forces one.
Each graph is stepped once from identical positions under both orders and on
both iteration paths (segment layout and direct gathers), and compared with
the FP64 oracle at the 1e-5 gates (1e-12 in FP64)."""
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


def _hubbed_path(n=20000, every=4):
    """A path 0-1-...-(n-1) plus a hub joined to every `every`-th vertex: most
    edges are short, and the hub's 2-hop row is far longer than 8192."""
    src = list(range(n - 1)) + [n] * len(range(0, n, every))
    dst = list(range(1, n)) + list(range(0, n, every))
    return inputs.to_csr(n + 1, src, dst)


CASES = [
    ("ws4000_k3", lambda: inputs.watts_strogatz(4000, 6, 0.1, seed=5), 3),
    ("rmat12_k2", lambda: inputs.rmat(12, 4, 0.57, 0.19, 0.19, seed=3), 2),
    ("grid32_k2", lambda: inputs.grid_graph(32, 32), 2),
    ("star300_k2", lambda: inputs.star_graph(300), 2),
    ("hubbed_path_k2", _hubbed_path, 2),
]


@pytest.mark.parametrize("path", ["segment", "direct"])
@pytest.mark.parametrize("order", ["degree", "caller"])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_order_step_parity(G, case, order, path, monkeypatch):
    import torch
    monkeypatch.setenv("GILA_ORDER", order)
    if path == "direct":
        monkeypatch.setenv("GILA_PATH", "direct")
    name, make, k = next(c for c in CASES if c[0] == case)
    g = make()
    print(f"order {name} {order} {path}", flush=True)
    rp, ci = G.to_device_csr(g)
    kh = G.build_khop(rp, ci, k)
    optr, oidx = oracle_rows(g, k)
    for prec, tol in ((G.FP32_KAHAN, 1e-5), (G.FP64, 1e-12)):
        x0 = inputs.uniform_positions(g.n, seed=21, width=1200.0)
        if prec != G.FP64:
            x0 = x0.astype(np.float32).astype(np.float64)
        params = G.LayoutParams(temperature=np.array([25.0]), ideal_length=48.0, precision=prec)
        pos = torch.from_numpy(x0).to(dtype=G.position_dtype(prec), device="cuda").contiguous()
        F = torch.zeros((g.n, 2), dtype=torch.float64, device="cuda")
        D = torch.zeros((g.n, 2), dtype=torch.float64, device="cuda")
        G.step(kh, params, 0, pos, F, D)
        xo, Fo, _, _ = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, 48.0, 25.0, x0)
        assert rel_l2(F.cpu().numpy(), Fo) <= tol, (name, order, path, prec)
        assert pos_err(pos.double().cpu().numpy(), xo) <= tol, (name, order, path, prec)
    # the lists are the same whatever the order
    ptr, idx = kh.export()
    assert np.array_equal(ptr, optr) and np.array_equal(idx, oidx)
    kh.free()
