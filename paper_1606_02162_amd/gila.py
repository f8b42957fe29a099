"""Thin ctypes binding of libgila (``include/gila.h``).

Argument marshalling only: every step of the layout runs in the library's HIP
kernels.  Device buffers are torch tensors on a ROCm device (torch is used for
device memory and the current stream only); host buffers are numpy arrays.
Importing this module loads ``libgila.so`` and raises if it has not been
built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GILA_LIBRARY") or os.path.join(_HERE, "libgila.so")

GILA_OK = 0
GILA_EINVAL = -1
GILA_ENOMEM = -2
GILA_EDEVICE = -3
GILA_EAGAIN = -4
GILA_ECANCELED = -5
GILA_EUNSUPPORTED = -6
GILA_ENONFINITE = -7

FP64 = 0
FP32 = 1
FP32_KAHAN = 2

PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32_kahan": FP32_KAHAN}

MODEL_FR = 0      # p = 2, q = 1
MODEL_LINLOG = 1  # p = 0, q = 1
MODEL_PQ = 2      # exponents given explicitly


class GilaError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {code})")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("ideal_length", ctypes.c_double),
                ("iterations", ctypes.c_int32), ("temperature", ctypes.POINTER(ctypes.c_double)),
                ("stop_fraction", ctypes.c_double), ("stop_displacement", ctypes.c_double),
                ("force_model", ctypes.c_int32), ("force_p", ctypes.c_int32),
                ("force_q", ctypes.c_int32)]


# numpy mirrors of gila_csr and gila_params, for marshalling thousands at once
CSR_DTYPE = np.dtype({"names": ["n", "nnz", "row_ptr", "col_idx"],
                      "formats": [np.int32, np.int64, np.uint64, np.uint64],
                      "offsets": [Csr.n.offset, Csr.nnz.offset, Csr.row_ptr.offset,
                                  Csr.col_idx.offset],
                      "itemsize": ctypes.sizeof(Csr)})
PARAMS_DTYPE = np.dtype({"names": ["precision", "ideal_length", "iterations", "temperature",
                                   "stop_fraction", "stop_displacement", "force_model",
                                   "force_p", "force_q"],
                         "formats": [np.int32, np.float64, np.int32, np.uint64, np.float64,
                                     np.float64, np.int32, np.int32, np.int32],
                         "offsets": [_Params.precision.offset, _Params.ideal_length.offset,
                                     _Params.iterations.offset, _Params.temperature.offset,
                                     _Params.stop_fraction.offset,
                                     _Params.stop_displacement.offset,
                                     _Params.force_model.offset, _Params.force_p.offset,
                                     _Params.force_q.offset],
                         "itemsize": ctypes.sizeof(_Params)})


METRIC_CROSSINGS = 1
METRIC_LENGTHS = 2
METRIC_SIMILARITY = 4


class Metrics(ctypes.Structure):
    _fields_ = [("edges", ctypes.c_int64), ("crossings", ctypes.c_int64),
                ("edge_length_mean", ctypes.c_double), ("edge_length_std", ctypes.c_double),
                ("similarity", ctypes.c_double), ("gabriel_edges", ctypes.c_int64)]

    @property
    def crossings_per_edge(self) -> float:
        """CRE: crossings divided by the number of edges (0 without edges)."""
        return self.crossings / self.edges if self.edges else 0.0

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("iterations_run", ctypes.c_int32), ("stopped", ctypes.c_int32),
                ("moved", ctypes.c_int64), ("max_disp", ctypes.c_double),
                ("energy", ctypes.c_double), ("coincident", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libgila.so not built at {path}: run `python -m paper_1606_02162_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "gila_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "gila_last_error": (ctypes.c_char_p, []),
        "gila_version": (ctypes.c_int, []),
        "gila_release_cached_memory": (i64, []),
        "gila_build_khop": (ctypes.c_int, [P(Csr), i32, vp, P(vp)]),
        "gila_khop_info": (ctypes.c_int, [vp, P(i32), P(i32), P(i64), P(i32), P(i64)]),
        "gila_khop_export": (ctypes.c_int, [vp, vp, vp]),
        "gila_khop_export_rows": (ctypes.c_int, [vp, i64, vp, vp, vp]),
        "gila_khop_free": (None, [vp]),
        "gila_khop_order": (ctypes.c_int, [vp, vp]),
        "gila_khop_set_mass": (ctypes.c_int, [vp, vp, vp]),
        "gila_prune": (ctypes.c_int, [P(Csr), vp, P(vp)]),
        "gila_pruned_info": (ctypes.c_int, [vp, P(i32), P(i64), P(i32), P(i32), P(i64)]),
        "gila_pruned_graph": (ctypes.c_int, [vp, P(Csr), P(vp)]),
        "gila_pruned_export": (ctypes.c_int, [vp, vp, vp, vp]),
        "gila_pruned_gather": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "gila_reinsert": (ctypes.c_int, [vp, dbl, i32, vp, vp, vp]),
        "gila_pruned_free": (None, [vp]),
        "gila_layout_pruned": (ctypes.c_int, [P(Csr), i32, P(_Params), vp, vp, P(Stats)]),
        "gila_components": (ctypes.c_int, [P(Csr), vp, P(i32), vp]),
        "gila_components_noalloc": (ctypes.c_int, [P(Csr), vp, P(i32), vp]),
        "gila_drawing_metrics": (ctypes.c_int, [P(Csr), i32, vp, i32, vp, P(Metrics), vp, vp]),
        "gila_pack_components": (ctypes.c_int, [i32, vp, dbl, i32, vp, vp]),
        "gila_layout_components": (ctypes.c_int, [P(Csr), i32, P(_Params), vp, vp, P(i32), vp]),
        "gila_init_positions": (ctypes.c_int, [i32, u64, dbl, dbl, i32, vp, vp]),
        "gila_paper_schedule": (ctypes.c_int, [dbl, dbl, dbl, i32, vp]),
        "gila_linear_schedule": (ctypes.c_int, [dbl, i32, vp]),
        "gila_step": (ctypes.c_int, [vp, P(_Params), i32, vp, vp, vp, vp, P(Stats)]),
        "gila_enable_history": (ctypes.c_int, [vp, i32, vp]),
        "gila_history": (ctypes.c_int, [vp, i32, i32, vp, vp]),
        "gila_run": (ctypes.c_int, [vp, P(_Params), i32, i32, vp, vp, P(Stats)]),
        "gila_layout": (ctypes.c_int, [P(Csr), i32, P(_Params), vp, vp, P(Stats)]),
        "gila_time_iterations": (ctypes.c_int, [vp, P(_Params), i32, i32, vp, vp,
                                                P(ctypes.c_double)]),
        "gila_batch_build": (ctypes.c_int, [vp, i32, vp, vp, P(vp)]),
        "gila_batch_run": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "gila_batch_info": (ctypes.c_int, [vp, P(i32), P(i64), P(i64)]),
        "gila_batch_free": (None, [vp]),
        "gila_batch_latency": (ctypes.c_int, [vp, vp]),
        "gila_batch_export": (ctypes.c_int, [vp, i32, vp, vp]),
        "gila_batch_plan": (ctypes.c_int, [vp, vp, vp]),
        "gila_batch_set_plan": (ctypes.c_int, [vp, vp]),
        "gila_batch_tune": (ctypes.c_int, [vp, i32, vp, vp]),
        "gila_layout_batch": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp]),
        "gila_server_create": (ctypes.c_int, [i32, i64, i32, P(vp)]),
        "gila_server_config": (ctypes.c_int, [vp, ctypes.c_char_p, i64]),
        "gila_job_latency": (ctypes.c_int, [vp, u64, P(dbl), P(dbl)]),
        "gila_submit": (ctypes.c_int, [vp, P(Csr), i32, P(_Params), vp, P(u64)]),
        "gila_poll": (ctypes.c_int, [vp, u64, vp, P(Stats)]),
        "gila_wait": (ctypes.c_int, [vp, u64, vp, P(Stats)]),
        "gila_cancel": (ctypes.c_int, [vp, u64]),
        "gila_server_info": (ctypes.c_int, [vp, P(i64), P(i64), P(i32), P(i64)]),
        "gila_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def lib() -> ctypes.CDLL:
    return _lib


def _check(rc: int, where: str):
    if rc != GILA_OK:
        msg = _lib.gila_last_error().decode(errors="replace") or _lib.gila_strerror(rc).decode()
        raise GilaError(rc, where, msg)


def _stream(stream=None) -> int:
    if stream is not None:
        return int(getattr(stream, "cuda_stream", stream))
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _addr(arr):
    return ctypes.cast(arr, ctypes.c_void_p)


def _ptr(t) -> int:
    if t is None:
        return 0
    return int(t.data_ptr())


# ---------------------------------------------------------------- schedules
# The paper's ideal edge length d = 20 + sqrt(800) (Section 5.1).
PAPER_IDEAL_LENGTH = 48.2842712474619
def release_cached_memory() -> int:
    """Returns the library's cached device blocks to the device; the bytes returned."""
    return int(lib().gila_release_cached_memory())


def paper_schedule(n_vertices: float, aspect: float, ideal_length: float,
                   iterations: int) -> np.ndarray:
    """Cap of Section 5.1 (``gila_paper_schedule``): sqrt((n / a) d) 0.93^h,
    h = 0 .. iterations-1."""
    t = np.zeros(max(int(iterations), 1), dtype=np.float64)
    _check(_lib.gila_paper_schedule(float(n_vertices), float(aspect), float(ideal_length),
                                    int(iterations), t.ctypes.data), "gila_paper_schedule")
    return t[: int(iterations)]


def linear_schedule(t0: float, iterations: int) -> np.ndarray:
    """``gila_linear_schedule``: t0 - t0 h / iterations, h = 0 .. iterations-1
    (t0 down to t0 / iterations)."""
    t = np.zeros(max(int(iterations), 1), dtype=np.float64)
    _check(_lib.gila_linear_schedule(float(t0), int(iterations), t.ctypes.data),
           "gila_linear_schedule")
    return t[: int(iterations)]


# ---------------------------------------------------------------- params
@dataclass
class LayoutParams:
    temperature: np.ndarray
    ideal_length: float = PAPER_IDEAL_LENGTH
    precision: int = FP32_KAHAN
    stop_fraction: float = 0.0
    stop_displacement: float = 0.01
    force_model: int = MODEL_FR
    force_p: int = 2
    force_q: int = 1
    _keep: list = field(default_factory=list, repr=False)

    @property
    def iterations(self) -> int:
        return int(np.asarray(self.temperature).size)

    def as_struct(self) -> _Params:
        t = np.ascontiguousarray(self.temperature, dtype=np.float64)
        self._keep = [t]
        p = _Params()
        p.precision = int(self.precision)
        p.ideal_length = float(self.ideal_length)
        p.iterations = int(t.size)
        p.temperature = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if t.size else None
        p.stop_fraction = float(self.stop_fraction)
        p.stop_displacement = float(self.stop_displacement)
        p.force_model = int(self.force_model)
        p.force_p = int(self.force_p)
        p.force_q = int(self.force_q)
        return p


def position_dtype(precision: int):
    import torch
    return torch.float64 if precision == FP64 else torch.float32


def make_csr(row_ptr, col_idx, n: int | None = None) -> Csr:
    """CSR descriptor over torch device tensors (or numpy host arrays)."""
    if n is None:
        n = int(row_ptr.shape[0]) - 1
    c = Csr()
    c.n = n
    c.nnz = int(col_idx.shape[0])
    if isinstance(row_ptr, np.ndarray):
        c.row_ptr = row_ptr.ctypes.data
        c.col_idx = col_idx.ctypes.data
    else:
        c.row_ptr = _ptr(row_ptr)
        c.col_idx = _ptr(col_idx)
    return c


def to_device_csr(graph, device="cuda"):
    """Upload an ``inputs.Graph`` to device tensors (row_ptr int64, col_idx int32)."""
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(graph.row_ptr, dtype=np.int64)).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(graph.col_idx, dtype=np.int32)).to(device)
    return rp, ci


# ---------------------------------------------------------------- k-hop handle
class KHop:
    """Device k-neighbourhood lists of one graph (gila_build_khop)."""

    def __init__(self, row_ptr, col_idx, k: int, stream=None, _csr: Csr | None = None):
        self._h = ctypes.c_void_p()
        self._csr = _csr if _csr is not None else make_csr(row_ptr, col_idx)
        _check(_lib.gila_build_khop(ctypes.byref(self._csr), int(k), _stream(stream),
                                    ctypes.byref(self._h)), "gila_build_khop")

    @classmethod
    def from_csr(cls, csr: Csr, k: int, stream=None) -> "KHop":
        """Build from a device CSR descriptor (e.g. ``Pruned.graph()``)."""
        return cls(None, None, k, stream, _csr=csr)

    def set_mass(self, mass=None, stream=None):
        """Weights of the repulsion each vertex exerts (gila_khop_set_mass):
        a float64 device tensor of n entries, a raw device address, or None
        for unit weights."""
        addr = mass if isinstance(mass, int) else _ptr(mass)
        _check(_lib.gila_khop_set_mass(self._h, addr, _stream(stream)), "gila_khop_set_mass")

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, k, na = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        P, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.gila_khop_info(self._h, ctypes.byref(n), ctypes.byref(k), ctypes.byref(P),
                                   ctypes.byref(na), ctypes.byref(b)), "gila_khop_info")
        return {"n": n.value, "k": k.value, "total_pairs": P.value, "n_active": na.value,
                "device_bytes": b.value}

    def enable_history(self, capacity: int, stream=None):
        """Record the statistics of iterations 0 .. capacity-1 of later runs
        on this handle (gila_enable_history; 0 frees the table)."""
        _check(_lib.gila_enable_history(self._h, int(capacity), _stream(stream)),
               "gila_enable_history")
        self._hist_cap = int(capacity)

    def history(self, h0: int = 0, count: int | None = None, stream=None) -> np.ndarray:
        """Rows [h0, h0 + count) of the per-iteration statistics as float64
        (count, 4): energy, max displacement, moved, coincident; NaN for
        iterations not run (gila_history)."""
        if count is None:
            count = getattr(self, "_hist_cap", 0) - h0
        rows = np.zeros((max(count, 0), 4), dtype=np.float64)
        _check(_lib.gila_history(self._h, int(h0), int(count), rows.ctypes.data if count > 0 else None,
                                 _stream(stream)), "gila_history")
        return rows

    def export(self):
        inf = self.info()
        ptr = np.zeros(inf["n"] + 1, dtype=np.int64)
        idx = np.zeros(max(inf["total_pairs"], 1), dtype=np.int32)
        _check(_lib.gila_khop_export(self._h, ptr.ctypes.data, idx.ctypes.data),
               "gila_khop_export")
        return ptr, idx[: inf["total_pairs"]]

    def export_rows(self, verts):
        v = np.ascontiguousarray(verts, dtype=np.int32)
        ptr = np.zeros(v.size + 1, dtype=np.int64)
        _check(_lib.gila_khop_export_rows(self._h, v.size, v.ctypes.data, ptr.ctypes.data, None),
               "gila_khop_export_rows")
        idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
        _check(_lib.gila_khop_export_rows(self._h, v.size, v.ctypes.data, ptr.ctypes.data,
                                          idx.ctypes.data), "gila_khop_export_rows")
        return ptr, idx[: int(ptr[-1])]

    def order(self) -> np.ndarray:
        """Caller id of each internal position (gila_khop_order)."""
        out = np.zeros(max(self.info()["n"], 1), dtype=np.int32)
        _check(_lib.gila_khop_order(self._h, out.ctypes.data), "gila_khop_order")
        return out[: self.info()["n"]]

    def free(self):
        if self._h:
            _lib.gila_khop_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_khop(row_ptr, col_idx, k: int, stream=None) -> KHop:
    return KHop(row_ptr, col_idx, k, stream)


def init_positions(n: int, seed: int, width: float, height: float, precision: int, out,
                   stream=None):
    _check(_lib.gila_init_positions(int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, float(width),
                                    float(height), int(precision), _ptr(out), _stream(stream)),
           "gila_init_positions")
    return out


def step(kh: KHop, params: LayoutParams, h: int, pos, force=None, disp=None,
         stream=None) -> Stats:
    st = Stats()
    p = params.as_struct()
    _check(_lib.gila_step(kh.handle, ctypes.byref(p), int(h), _ptr(pos), _ptr(force), _ptr(disp),
                          _stream(stream), ctypes.byref(st)), "gila_step")
    return st


def run(kh: KHop, params: LayoutParams, pos, start_h: int = 0, end_h: int | None = None,
        stream=None) -> Stats:
    st = Stats()
    p = params.as_struct()
    if end_h is None:
        end_h = params.iterations
    _check(_lib.gila_run(kh.handle, ctypes.byref(p), int(start_h), int(end_h), _ptr(pos),
                         _stream(stream), ctypes.byref(st)), "gila_run")
    return st


def time_iterations(kh: KHop, params: LayoutParams, pos, h: int = 0, reps: int = 10,
                    stream=None, with_mode: bool = False):
    """Average (force kernel, rest of the iteration) milliseconds over `reps`
    iterations starting at h, run as gila_run runs them between HIP events,
    the force kernel's share from its own start/end stamps on the device wall
    clock (gila_time_iterations).  With ``with_mode`` a third value tells
    whether the iterations ran as a graph replay (True) or, when capture was
    refused, eagerly (False)."""
    ms = (ctypes.c_double * 3)()
    p = params.as_struct()
    _check(_lib.gila_time_iterations(kh.handle, ctypes.byref(p), int(h), int(reps), _ptr(pos),
                                     _stream(stream), ms), "gila_time_iterations")
    if with_mode:
        return float(ms[0]), float(ms[1]), bool(ms[2] == 1.0)
    return float(ms[0]), float(ms[1])


def layout(row_ptr, col_idx, k: int, params: LayoutParams, pos, stream=None) -> Stats:
    st = Stats()
    csr = make_csr(row_ptr, col_idx)
    p = params.as_struct()
    _check(_lib.gila_layout(ctypes.byref(csr), int(k), ctypes.byref(p), _ptr(pos),
                            _stream(stream), ctypes.byref(st)), "gila_layout")
    return st


# ---------------------------------------------------------------- pruning
class Pruned:
    """Degree-one vertices removed from a device graph (gila_prune)."""

    def __init__(self, row_ptr, col_idx, stream=None, _csr: Csr | None = None):
        self._h = ctypes.c_void_p()
        self._csr = _csr if _csr is not None else make_csr(row_ptr, col_idx)
        self.n = self._csr.n
        _check(_lib.gila_prune(ctypes.byref(self._csr), _stream(stream), ctypes.byref(self._h)),
               "gila_prune")

    def info(self) -> dict:
        nk, npr, na = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nnz, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.gila_pruned_info(self._h, ctypes.byref(nk), ctypes.byref(nnz),
                                     ctypes.byref(npr), ctypes.byref(na), ctypes.byref(b)),
               "gila_pruned_info")
        return {"n_kept": nk.value, "nnz_kept": nnz.value, "n_pruned": npr.value,
                "n_with_leaves": na.value, "device_bytes": b.value}

    def graph(self):
        """(Csr of the pruned graph, device address of its float64 weights);
        both live as long as this handle."""
        csr = Csr()
        m = ctypes.c_void_p()
        _check(_lib.gila_pruned_graph(self._h, ctypes.byref(csr), ctypes.byref(m)),
               "gila_pruned_graph")
        return csr, int(m.value or 0)

    def export(self):
        """Host (anchor, leaves, new_id), each int32[n] in original ids."""
        a = np.zeros(max(self.n, 1), dtype=np.int32)
        lv = np.zeros(max(self.n, 1), dtype=np.int32)
        ni = np.zeros(max(self.n, 1), dtype=np.int32)
        _check(_lib.gila_pruned_export(self._h, a.ctypes.data, lv.ctypes.data, ni.ctypes.data),
               "gila_pruned_export")
        return a[: self.n], lv[: self.n], ni[: self.n]

    def gather(self, precision: int, pos_all, pos_kept, stream=None):
        _check(_lib.gila_pruned_gather(self._h, int(precision), _ptr(pos_all), _ptr(pos_kept),
                                       _stream(stream)), "gila_pruned_gather")
        return pos_kept

    def reinsert(self, ideal_length: float, precision: int, pos_kept, pos_all, stream=None):
        _check(_lib.gila_reinsert(self._h, float(ideal_length), int(precision), _ptr(pos_kept),
                                  _ptr(pos_all), _stream(stream)), "gila_reinsert")
        return pos_all

    def free(self):
        if self._h:
            _lib.gila_pruned_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def prune(row_ptr, col_idx, stream=None) -> Pruned:
    return Pruned(row_ptr, col_idx, stream)


def layout_pruned(row_ptr, col_idx, k: int, params: LayoutParams, pos, stream=None) -> Stats:
    """Prune, lay out the pruned graph with leaf-weighted repulsion, reinsert
    (gila_layout_pruned); pos holds every vertex, in and out."""
    st = Stats()
    csr = make_csr(row_ptr, col_idx)
    p = params.as_struct()
    _check(_lib.gila_layout_pruned(ctypes.byref(csr), int(k), ctypes.byref(p), _ptr(pos),
                                   _stream(stream), ctypes.byref(st)), "gila_layout_pruned")
    return st


# ---------------------------------------------------------------- components
def components(row_ptr, col_idx, stream=None):
    """(label int32 device tensor: smallest id of each vertex's component,
    number of components) -- gila_components."""
    import torch
    csr = make_csr(row_ptr, col_idx)
    label = torch.empty(max(csr.n, 1), dtype=torch.int32, device=row_ptr.device)
    c = ctypes.c_int32()
    _check(_lib.gila_components(ctypes.byref(csr), _ptr(label), ctypes.byref(c), _stream(stream)),
           "gila_components")
    return label[: csr.n], c.value


def components_noalloc(row_ptr, col_idx, label, stream=None) -> int:
    """gila_components_noalloc: the labels of gila_components written into the
    caller's int32 device tensor ``label`` (n entries) with no device
    allocation by the library; returns the number of components."""
    csr = make_csr(row_ptr, col_idx)
    c = ctypes.c_int32()
    _check(_lib.gila_components_noalloc(ctypes.byref(csr), _ptr(label), ctypes.byref(c),
                                        _stream(stream)), "gila_components_noalloc")
    return c.value


def pack_components(label, gap: float, precision: int, pos, stream=None):
    """Pack the components' drawings in place (gila_pack_components)."""
    _check(_lib.gila_pack_components(int(label.shape[0]), _ptr(label), float(gap), int(precision),
                                     _ptr(pos), _stream(stream)), "gila_pack_components")
    return pos


def layout_components(row_ptr, col_idx, k: int, params: LayoutParams, pos, iterations=None,
                      stream=None):
    """Lay out every component alone with its own cap and halting rule, then
    pack (gila_layout_components).  The caps are the components' own:
    params.temperature only gives the iteration count unless `iterations` is
    set.  Returns (components, int32[n] iterations run by each vertex's
    component)."""
    csr = make_csr(row_ptr, col_idx)
    p = params.as_struct()
    if iterations is not None:
        p.iterations = int(iterations)
        p.temperature = None
    c = ctypes.c_int32()
    runs = np.zeros(max(csr.n, 1), dtype=np.int32)
    _check(_lib.gila_layout_components(ctypes.byref(csr), int(k), ctypes.byref(p), _ptr(pos),
                                       _stream(stream), ctypes.byref(c), runs.ctypes.data),
           "gila_layout_components")
    return c.value, runs[: csr.n]


# ---------------------------------------------------------------- quality metrics
def drawing_metrics(row_ptr, col_idx, precision: int, pos, what: int = 7, edge_crossings=None,
                    jaccard=None, stream=None) -> Metrics:
    """Crossings, edge length mean / deviation and Gabriel similarity of a
    drawing (gila_drawing_metrics); edge_crossings (int64 device tensor [m])
    and jaccard (float64 device tensor [n]) are optional per-edge and
    per-vertex outputs."""
    csr = make_csr(row_ptr, col_idx)
    out = Metrics()
    _check(_lib.gila_drawing_metrics(ctypes.byref(csr), int(precision), _ptr(pos), int(what),
                                     _stream(stream), ctypes.byref(out), _ptr(edge_crossings),
                                     _ptr(jaccard)), "gila_drawing_metrics")
    return out


# ---------------------------------------------------------------- batches
class Batch:
    """Many graphs' k-hop lists in one segmented handle (gila_batch_build).

    ``graphs`` is a list of (row_ptr, col_idx) device tensor pairs, ``k`` a
    list of ints (or one int for all)."""

    def __init__(self, graphs, k, stream=None, _csr=None):
        if _csr is None:
            count = len(graphs)
            csr = np.zeros(max(count, 1), dtype=CSR_DTYPE)
            for i, (rp, ci) in enumerate(graphs):
                c = make_csr(rp, ci)
                csr[i] = (c.n, c.nnz, c.row_ptr or 0, c.col_idx or 0)
        else:
            csr, count = _csr, int(_csr.size)
        ks = np.full(max(count, 1), int(k), dtype=np.int32) if isinstance(k, int) else \
            np.ascontiguousarray(k, dtype=np.int32)
        self._csr, self._k, self.count = csr, ks, count
        self._h = ctypes.c_void_p()
        _check(_lib.gila_batch_build(csr.ctypes.data, count, ks.ctypes.data, _stream(stream),
                                     ctypes.byref(self._h)), "gila_batch_build")

    @classmethod
    def concatenated(cls, row_ptr_all, col_idx_all, n, nnz, k, stream=None):
        """Graphs given as one concatenation: graph i has n[i] vertices and
        nnz[i] adjacency entries; its row_ptr (n[i] + 1 entries, values from 0)
        and col_idx (its own ids) follow the previous graph's in the two
        device tensors."""
        n = np.ascontiguousarray(n, dtype=np.int64)
        nnz = np.ascontiguousarray(nnz, dtype=np.int64)
        rp_off = np.concatenate([[0], np.cumsum(n + 1)[:-1]]).astype(np.int64)
        ci_off = np.concatenate([[0], np.cumsum(nnz)[:-1]]).astype(np.int64)
        csr = np.zeros(max(n.size, 1), dtype=CSR_DTYPE)
        csr["n"][: n.size] = n
        csr["nnz"][: n.size] = nnz
        csr["row_ptr"][: n.size] = _ptr(row_ptr_all) + 8 * rp_off
        csr["col_idx"][: n.size] = _ptr(col_idx_all) + 4 * ci_off
        csr = csr[: n.size] if n.size else csr[:0]
        return cls(None, k, stream=stream, _csr=np.ascontiguousarray(csr))

    def info(self) -> dict:
        c, P, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.gila_batch_info(self._h, ctypes.byref(c), ctypes.byref(P), ctypes.byref(b)),
               "gila_batch_info")
        return {"count": c.value, "total_pairs": P.value, "device_bytes": b.value}

    def run(self, params, pos, stream=None):
        """params: list of LayoutParams (or one for all), or a BatchParams;
        pos: list of device tensors, or (one tensor, vertex offset of each
        graph) for graphs laid out one after another in it; updated in place.
        Returns a list of Stats."""
        if isinstance(params, BatchParams):
            structs = params.structs
        else:
            plist = params if isinstance(params, (list, tuple)) else [params] * self.count
            structs = (_Params * max(self.count, 1))()
            for i, p in enumerate(plist):
                structs[i] = p.as_struct()
        if isinstance(pos, tuple):
            t, voff = pos
            ptrs = np.ascontiguousarray(_ptr(t) + 2 * t.element_size() *
                                        np.asarray(voff, dtype=np.int64), dtype=np.uint64)
            paddr = ptrs.ctypes.data
        else:
            ptrs = (ctypes.c_void_p * max(self.count, 1))(*[_ptr(t) for t in pos])
            paddr = _addr(ptrs)
        saddr = structs.ctypes.data if isinstance(structs, np.ndarray) else _addr(structs)
        stats = (Stats * max(self.count, 1))()
        _check(_lib.gila_batch_run(self._h, saddr, paddr, _stream(stream), _addr(stats)),
               "gila_batch_run")
        return [stats[i] for i in range(self.count)]

    def export(self, graph: int, n: int):
        """k-hop lists of graph `graph` (n vertices) in its own ids: (ptr, idx)."""
        ptr = np.zeros(n + 1, dtype=np.int64)
        _check(_lib.gila_batch_export(self._h, graph, ptr.ctypes.data, None), "gila_batch_export")
        idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
        _check(_lib.gila_batch_export(self._h, graph, ptr.ctypes.data, idx.ctypes.data),
               "gila_batch_export")
        return ptr, idx[: int(ptr[-1])]

    def plan(self):
        """(lanes per vertex, row-length class) of every graph: gila_batch_plan."""
        lanes = np.zeros(max(self.count, 1), dtype=np.int32)
        cls = np.zeros(max(self.count, 1), dtype=np.int32)
        _check(_lib.gila_batch_plan(self._h, lanes.ctypes.data, cls.ctypes.data),
               "gila_batch_plan")
        return lanes[: self.count], cls[: self.count]

    def set_plan(self, lanes):
        """gila_batch_set_plan: lanes per vertex of every graph."""
        arr = np.ascontiguousarray(lanes, dtype=np.int32)
        if arr.size != self.count:
            raise ValueError("one lanes-per-vertex value per graph")
        _check(_lib.gila_batch_set_plan(self._h, arr.ctypes.data if arr.size else None),
               "gila_batch_set_plan")

    def tune(self, precision: int, stream=None) -> np.ndarray:
        """gila_batch_tune: times the choices per row-length class, sets the
        fastest in the plan; returns the table (8 classes, 0 = absent)."""
        table = np.zeros(8, dtype=np.int32)
        _check(_lib.gila_batch_tune(self._h, int(precision), _stream(stream), table.ctypes.data),
               "gila_batch_tune")
        return table

    def latency_ms(self) -> np.ndarray:
        """Per-graph completion time (ms) of the last run, from its first start."""
        out = np.zeros(max(self.count, 1), dtype=np.float64)
        _check(_lib.gila_batch_latency(self._h, out.ctypes.data), "gila_batch_latency")
        return out[: self.count]

    def free(self):
        if self._h:
            _lib.gila_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class BatchParams:
    """Parameters of every graph of a batch marshalled once: temperatures is a
    list of per-graph schedules; ideal_length, precision and the halting
    settings are shared."""

    def __init__(self, temperatures, ideal_length=PAPER_IDEAL_LENGTH,
                 precision=FP32_KAHAN, stop_fraction=0.0, stop_displacement=0.01):
        lens = np.array([len(t) for t in temperatures], dtype=np.int64)
        self._t = np.ascontiguousarray(np.concatenate(temperatures) if len(temperatures) else
                                       np.zeros(1), dtype=np.float64)
        off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        st = np.zeros(max(lens.size, 1), dtype=PARAMS_DTYPE)
        st["precision"] = int(precision)
        st["ideal_length"] = float(ideal_length)
        st["iterations"][: lens.size] = lens
        st["temperature"][: lens.size] = np.where(lens > 0, self._t.ctypes.data + 8 * off, 0)
        st["stop_fraction"] = float(stop_fraction)
        st["stop_displacement"] = float(stop_displacement)
        self.structs = st


def layout_batch(graphs, k, params, pos, stream=None):
    """Build, run and free a batch in one call (gila_layout_batch)."""
    count = len(graphs)
    ks = [int(k)] * count if isinstance(k, int) else [int(x) for x in k]
    csr = (Csr * max(count, 1))()
    for i, (rp, ci) in enumerate(graphs):
        csr[i] = make_csr(rp, ci)
    kk = (ctypes.c_int32 * max(count, 1))(*ks)
    plist = params if isinstance(params, (list, tuple)) else [params] * count
    structs = (_Params * max(count, 1))()
    for i, p in enumerate(plist):
        structs[i] = p.as_struct()
    ptrs = (ctypes.c_void_p * max(count, 1))(*[_ptr(t) for t in pos])
    stats = (Stats * max(count, 1))()
    _check(_lib.gila_layout_batch(_addr(csr), count, _addr(kk), _addr(structs), _addr(ptrs),
                                  _stream(stream), _addr(stats)), "gila_layout_batch")
    return [stats[i] for i in range(count)]


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching layout server (gila_server_*).  Jobs are host
    graphs (``inputs.Graph`` or any object with n, row_ptr, col_idx) with host
    initial positions (float64 [n, 2])."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, max_slots: int = 64):
        self._h = ctypes.c_void_p()
        _check(_lib.gila_server_create(int(device), int(budget_bytes), int(max_slots),
                                       ctypes.byref(self._h)), "gila_server_create")
        self._keep = {}

    def config(self, key: str, value: int):
        _check(_lib.gila_server_config(self._h, key.encode(), int(value)), "gila_server_config")

    def submit(self, graph, k: int, params: LayoutParams, init_pos) -> int:
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(graph.col_idx, dtype=np.int32)
        x = np.ascontiguousarray(init_pos, dtype=np.float64).reshape(-1)
        csr = make_csr(rp, ci, int(graph.n))
        p = params.as_struct()
        t = ctypes.c_uint64()
        _check(_lib.gila_submit(self._h, ctypes.byref(csr), int(k), ctypes.byref(p),
                                x.ctypes.data if x.size else None, ctypes.byref(t)),
               "gila_submit")
        self._keep[t.value] = int(graph.n)
        return t.value

    def poll(self, ticket: int):
        """(status, positions or None, Stats); status GILA_EAGAIN while running."""
        n = self._keep.get(ticket, 0)
        out = np.zeros((max(n, 1), 2), dtype=np.float64)
        st = Stats()
        rc = _lib.gila_poll(self._h, int(ticket), out.ctypes.data, ctypes.byref(st))
        if rc == GILA_EAGAIN:
            return rc, None, None
        self._keep.pop(ticket, None)
        return rc, (out[:n] if rc == GILA_OK else None), st

    def wait(self, ticket: int):
        n = self._keep.get(ticket, 0)
        out = np.zeros((max(n, 1), 2), dtype=np.float64)
        st = Stats()
        rc = _lib.gila_wait(self._h, int(ticket), out.ctypes.data, ctypes.byref(st))
        self._keep.pop(ticket, None)
        _check(rc, "gila_wait")
        return out[:n], st

    def cancel(self, ticket: int):
        _check(_lib.gila_cancel(self._h, int(ticket)), "gila_cancel")

    def latency(self, ticket: int):
        q, t = ctypes.c_double(), ctypes.c_double()
        _check(_lib.gila_job_latency(self._h, int(ticket), ctypes.byref(q), ctypes.byref(t)),
               "gila_job_latency")
        return q.value, t.value

    def info(self) -> dict:
        d, t, p, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib.gila_server_info(self._h, ctypes.byref(d), ctypes.byref(t), ctypes.byref(p),
                                     ctypes.byref(b)), "gila_server_info")
        return {"jobs_done": d.value, "ticks": t.value, "peak_resident": p.value,
                "bytes_reserved": b.value}

    def close(self):
        if self._h:
            _lib.gila_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
