"""Host-only checks of the C ABI: the built library loads, exports every
function that include/gila.h declares, and rejects bad arguments before any
device work (these calls never reach the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gila.h")
LIB = os.path.join(ROOT, "paper_1606_02162_amd", "libgila.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gila_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgila.so is not built; run `python -m paper_1606_02162_amd.build`")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("gila_build_khop", "gila_step", "gila_run", "gila_layout", "gila_submit",
                     "gila_poll", "gila_layout_batch", "gila_khop_export", "gila_prune",
                     "gila_reinsert", "gila_khop_set_mass", "gila_layout_pruned",
                     "gila_components", "gila_pack_components", "gila_layout_components",
                     "gila_drawing_metrics"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls(lib):
    lib.gila_strerror.restype = ctypes.c_char_p
    lib.gila_last_error.restype = ctypes.c_char_p
    assert lib.gila_version() >= 10000
    assert lib.gila_strerror(-1) == b"invalid argument or malformed graph"
    assert lib.gila_strerror(0) == b"ok"


def test_argument_validation_before_device_work():
    from paper_1606_02162_amd import gila
    L = gila.lib()
    out = ctypes.c_void_p()
    csr = gila.Csr()
    csr.n = 4
    csr.nnz = 2
    # k < 1
    assert L.gila_build_khop(ctypes.byref(csr), 0, None, ctypes.byref(out)) == gila.GILA_EINVAL
    assert b"k must be" in L.gila_last_error()
    # batch export without a batch
    ptr = (ctypes.c_int64 * 4)()
    assert L.gila_batch_export(None, 0, ptr, None) == gila.GILA_EINVAL
    # null graph / null out
    assert L.gila_build_khop(None, 2, None, ctypes.byref(out)) == gila.GILA_EINVAL
    assert L.gila_build_khop(ctypes.byref(csr), 2, None, None) == gila.GILA_EINVAL
    # null row_ptr with n > 0
    assert L.gila_build_khop(ctypes.byref(csr), 2, None, ctypes.byref(out)) == gila.GILA_EINVAL
    # negative n
    csr.n = -1
    assert L.gila_build_khop(ctypes.byref(csr), 2, None, ctypes.byref(out)) == gila.GILA_EINVAL
    # null handles
    assert L.gila_khop_info(None, None, None, None, None, None) == gila.GILA_EINVAL
    assert L.gila_run(None, None, 0, 0, None, None, None) == gila.GILA_EINVAL
    assert L.gila_step(None, None, 0, None, None, None, None, None) == gila.GILA_EINVAL
    assert L.gila_enable_history(None, 10, None) == gila.GILA_EINVAL
    assert L.gila_history(None, 0, 1, None, None) == gila.GILA_EINVAL
    # init positions: negative n, bad precision
    assert L.gila_init_positions(-1, 0, 1.0, 1.0, 1, None, None) == gila.GILA_EINVAL
    assert L.gila_init_positions(0, 0, 1.0, 1.0, 1, None, None) == gila.GILA_OK
    # pruning and weights: null graph / handles, bad k
    assert L.gila_prune(None, None, ctypes.byref(out)) == gila.GILA_EINVAL
    csr.n = 4
    assert L.gila_prune(ctypes.byref(csr), None, ctypes.byref(out)) == gila.GILA_EINVAL
    assert b"row_ptr is NULL" in L.gila_last_error()
    assert L.gila_prune(ctypes.byref(csr), None, None) == gila.GILA_EINVAL
    assert L.gila_pruned_info(None, None, None, None, None, None) == gila.GILA_EINVAL
    assert L.gila_pruned_graph(None, None, None) == gila.GILA_EINVAL
    assert L.gila_pruned_export(None, None, None, None) == gila.GILA_EINVAL
    assert L.gila_pruned_gather(None, 1, None, None, None) == gila.GILA_EINVAL
    assert L.gila_reinsert(None, 10.0, 1, None, None, None) == gila.GILA_EINVAL
    assert L.gila_khop_set_mass(None, None, None) == gila.GILA_EINVAL
    import numpy as np
    p = gila.LayoutParams(temperature=np.ones(2)).as_struct()
    st = gila.Stats()
    assert L.gila_layout_pruned(ctypes.byref(csr), 0, ctypes.byref(p), None, None,
                                ctypes.byref(st)) == gila.GILA_EINVAL
    assert b"k must be" in L.gila_last_error()
    # components: null graph, bad sizes, bad k
    assert L.gila_components(None, None, None, None) == gila.GILA_EINVAL
    assert L.gila_pack_components(-1, None, 1.0, 1, None, None) == gila.GILA_EINVAL
    assert L.gila_pack_components(4, None, 1.0, 1, None, None) == gila.GILA_EINVAL
    assert L.gila_layout_components(ctypes.byref(csr), 0, ctypes.byref(p), None, None, None,
                                    None) == gila.GILA_EINVAL
    # metrics: no output struct, bad precision
    mt = gila.Metrics()
    assert L.gila_drawing_metrics(ctypes.byref(csr), 1, None, 7, None, None, None,
                                  None) == gila.GILA_EINVAL
    assert L.gila_drawing_metrics(ctypes.byref(csr), 9, None, 7, None, ctypes.byref(mt), None,
                                  None) == gila.GILA_EINVAL


def test_params_validation():
    import numpy as np
    from paper_1606_02162_amd import gila
    L = gila.lib()
    csr = gila.Csr()
    csr.n = 2
    csr.nnz = 2
    bad = [
        gila.LayoutParams(temperature=np.ones(3), ideal_length=-1.0),
        gila.LayoutParams(temperature=np.array([1.0, -2.0])),
        gila.LayoutParams(temperature=np.ones(2), precision=7),
        gila.LayoutParams(temperature=np.array([1.0, float("nan")])),
        gila.LayoutParams(temperature=np.ones(2), stop_fraction=-0.1),
        gila.LayoutParams(temperature=np.ones(2), force_model=7),
        gila.LayoutParams(temperature=np.ones(2), force_model=gila.MODEL_PQ, force_p=9),
        gila.LayoutParams(temperature=np.ones(2), force_model=gila.MODEL_PQ, force_q=-1),
    ]
    st = gila.Stats()
    for p in bad:
        s = p.as_struct()
        rc = L.gila_layout(ctypes.byref(csr), 2, ctypes.byref(s), None, None, ctypes.byref(st))
        assert rc == gila.GILA_EINVAL, p


def test_schedules_match_closed_forms():
    import math
    import numpy as np
    from paper_1606_02162_amd import gila
    t = gila.linear_schedule(100.0, 100)
    assert np.array_equal(t, 100.0 - np.arange(100))
    d = 20 + math.sqrt(800)
    p = gila.paper_schedule(1000, 1.0, d, 10)
    assert abs(p[0] ** 2 - 1000 * d) < 1e-9
    assert np.allclose(p[1:] / p[:-1], 0.93, rtol=1e-14, atol=0)


def test_schedule_argument_checks_and_new_status():
    import numpy as np
    from paper_1606_02162_amd import gila
    L = gila.lib()
    L.gila_strerror.restype = ctypes.c_char_p
    t = np.zeros(4)
    assert L.gila_paper_schedule(0.0, 1.0, 10.0, 4, t.ctypes.data) == gila.GILA_EINVAL
    assert L.gila_paper_schedule(10.0, -1.0, 10.0, 4, t.ctypes.data) == gila.GILA_EINVAL
    assert L.gila_paper_schedule(10.0, 1.0, 10.0, 4, None) == gila.GILA_EINVAL
    assert L.gila_paper_schedule(10.0, 1.0, 10.0, 0, None) == gila.GILA_OK
    assert L.gila_linear_schedule(-1.0, 4, t.ctypes.data) == gila.GILA_EINVAL
    assert L.gila_linear_schedule(5.0, -1, t.ctypes.data) == gila.GILA_EINVAL
    # a non-square frame: n / a with a = height / width (Section 5.1)
    p = gila.paper_schedule(500, 2.0, 8.0, 3)
    assert abs(p[0] ** 2 - 500 / 2.0 * 8.0) < 1e-9 and abs(p[2] / p[0] - 0.93 ** 2) < 1e-15
    assert L.gila_strerror(gila.GILA_ENONFINITE) == b"non-finite force"
