"""gila_components_noalloc (the entry point for callers that cannot allocate
device memory) against gila_components through the C ABI: the same labels
bit for bit and the same count, on two calls in a row with the second input
smaller than the first (the library's fixed scratch keeps the last call's
contents, so what must start at zero has to be cleared), and the same
argument and graph checks."""
import ctypes

import numpy as np
import pytest

from gpu_common import require_gpu
from paper_1606_02162_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    require_gpu()
    from paper_1606_02162_amd import gila
    return gila


def _union(*graphs):
    us, vs, off = [], [], 0
    for g in graphs:
        e = g.edges()
        us.append(e[:, 0] + off)
        vs.append(e[:, 1] + off)
        off += g.n
    return inputs.to_csr(off, np.concatenate(us), np.concatenate(vs), name="union")


def _shuffled(g, seed):
    p = np.random.default_rng(seed).permutation(g.n)
    e = g.edges()
    return inputs.to_csr(g.n, p[e[:, 0]], p[e[:, 1]], name=g.name + "_shuffled")


def _many(seed):
    rng = np.random.default_rng(seed)
    parts = [inputs.random_tree_plus_edges(int(s), int(s) // 3, seed=int(s) + seed)
             for s in rng.integers(2, 400, 80)]
    parts += [inputs.path_graph(2)] * 7 + [inputs.to_csr(50, [], [])]
    parts.append(inputs.barabasi_albert(5000, 2, seed=seed))
    return _shuffled(_union(*parts), seed)


def _both(G, g):
    import torch
    rp, ci = G.to_device_csr(g)
    ref_label, ref_count = G.components(rp, ci)
    label = torch.full((max(g.n, 1),), -7, dtype=torch.int32, device="cuda")
    count = G.components_noalloc(rp, ci, label[: g.n])
    return label[: g.n].cpu().numpy(), count, ref_label.cpu().numpy(), ref_count


def test_noalloc_matches_components_on_consecutive_calls(G):
    big = [inputs.rmat(16, 4, 0.57, 0.19, 0.19, seed=3), _many(2)]
    small = [_many(5), inputs.grid_graph(9, 7), inputs.to_csr(6, [0, 2], [1, 3]),
             inputs.to_csr(3, [], [])]
    for first, second in zip(big * 2, small):
        assert second.n < first.n
        for g in (first, second):
            print(f"noalloc {g.name} n={g.n}", flush=True)
            got, c, ref, rc = _both(G, g)
            assert c == rc, g.name
            assert np.array_equal(got, ref), g.name


def test_noalloc_rejects_malformed_graphs(G):
    import torch
    L = G.lib()
    label = torch.zeros(4, dtype=torch.int32, device="cuda")
    cases = [([0, 1, 2, 3, 3], [1, 0, 3]),     # odd nnz, asymmetric
             ([0, 2, 1, 2, 2], [1, 0]),        # row_ptr decreases
             ([1, 1, 2, 2, 2], [1, 0]),        # row_ptr[0] != 0
             ([0, 1, 2, 2, 2], [1, 1]),        # asymmetric / self-loop
             ([0, 1, 2, 2, 2], [9, 0])]        # column out of range
    for rp_h, ci_h in cases:
        rp = torch.tensor(rp_h, dtype=torch.int64, device="cuda")
        ci = torch.tensor(ci_h, dtype=torch.int32, device="cuda")
        csr = G.make_csr(rp, ci, n=4)
        cnt = ctypes.c_int32()
        rc = L.gila_components_noalloc(ctypes.byref(csr), label.data_ptr(), ctypes.byref(cnt),
                                       G._stream())
        assert rc == G.GILA_EINVAL, (rp_h, ci_h, rc)
    # after the refusals a valid call still gives the right labels
    g = inputs.to_csr(4, [0, 2], [1, 3])
    got, c, ref, rc = _both(G, g)
    assert c == rc == 2 and np.array_equal(got, ref)
    # no label buffer for a non-empty graph
    rp, ci = G.to_device_csr(g)
    csr = G.make_csr(rp, ci)
    assert L.gila_components_noalloc(ctypes.byref(csr), None, None, G._stream()) == G.GILA_EINVAL


def test_noalloc_empty_graph(G):
    import torch
    g = inputs.to_csr(0, [], [])
    rp, ci = G.to_device_csr(g)
    label = torch.empty(0, dtype=torch.int32, device="cuda")
    assert G.components_noalloc(rp, ci, label) == 0
