"""FP64 CPU oracle of GiLA's k-hop Fruchterman-Reingold layout.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here, and this
package imports nothing from the product path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, sequential sums in
ascending neighbour id; OpenMP only splits vertices across threads).  This
module compiles it with gcc and wraps it with ctypes and numpy.

Passages followed (Arleo, Didimo, Liotta, Montecchiani, "A Distributed
Force-Directed Algorithm on Giraph: Design and Experiments"):
  * Section 3.1, force equation and magnitudes ||f^a|| = delta^p/d,
    ||f^r|| = d^2/delta^q with p = 2, q = 1;
  * Section 4.5, the k-neighbourhood N_v(k), adjacent vertices receiving both
    forces, and the synchronous coordinate update;
  * Section 5.1, the cap schedule sqrt((n/a) d) 0.93^h and the halting rule.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class _IterStats(ctypes.Structure):
    _fields_ = [("moved", ctypes.c_int64), ("max_disp", ctypes.c_double),
                ("energy", ctypes.c_double), ("coincident", ctypes.c_int64)]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    lib.orc_khop_count.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int32, ctypes.c_int64,
                                   vp, _i64p]
    lib.orc_khop_fill.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int32, ctypes.c_int64,
                                  vp, _i64p, _i32p]
    lib.orc_forces.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int64, vp, _i64p, _i32p,
                               ctypes.c_double, _f64p, _f64p, ctypes.POINTER(ctypes.c_int64)]
    lib.orc_cap.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _f64p]
    lib.orc_step.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, _f64p, _f64p, _f64p,
                             ctypes.POINTER(_IterStats)]
    lib.orc_layout.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, ctypes.c_double,
                               _f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_double, _f64p, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(_IterStats)]
    lib.orc_paper_schedule.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, _f64p]
    lib.orc_linear_schedule.argtypes = [ctypes.c_double, ctypes.c_int32, _f64p]
    for f in ("orc_khop_count", "orc_khop_fill", "orc_forces", "orc_cap", "orc_step",
              "orc_layout"):
        getattr(lib, f).restype = ctypes.c_int
    lib.orc_paper_schedule.restype = None
    lib.orc_linear_schedule.restype = None
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _csr(row_ptr, col_idx):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col_idx, dtype=np.int32))


def _verts(verts):
    if verts is None:
        return None, None
    arr = np.ascontiguousarray(verts, dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def khop(n: int, row_ptr, col_idx, k: int, verts=None):
    """k-neighbourhood rows N_v(k) (Section 4.5), v excluded, ascending.

    Returns (ptr int64[count+1], idx int32[total]) for verts (default: all
    vertices in order).
    """
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    varr, vptr = _verts(verts)
    count = n if varr is None else varr.size
    sizes = np.zeros(max(count, 1), dtype=np.int64)
    _check(lib.orc_khop_count(n, rp, ci, k, count, vptr, sizes), "khop_count")
    ptr = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(sizes[:count], out=ptr[1:])
    idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
    _check(lib.orc_khop_fill(n, rp, ci, k, count, vptr, ptr, idx), "khop_fill")
    return ptr, idx[: int(ptr[-1])]


def forces(n: int, row_ptr, col_idx, kptr, kidx, d: float, pos, verts=None):
    """F_v for verts (Section 3.1 with N_v(k) repulsion, Section 4.5).

    ``kptr``/``kidx`` hold the rows of exactly the vertices in ``verts``
    (all vertices when verts is None).  ``pos`` is float64[n, 2].
    Returns (F float64[count, 2], coincident pair count).
    """
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    varr, vptr = _verts(verts)
    count = n if varr is None else varr.size
    p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    F = np.zeros(2 * max(count, 1), dtype=np.float64)
    coinc = ctypes.c_int64(0)
    _check(lib.orc_forces(n, rp, ci, count, vptr, kp, ki, float(d), p, F, ctypes.byref(coinc)),
           "forces")
    return F[: 2 * count].reshape(count, 2), int(coinc.value)


def cap(F, t: float):
    """Delta = F min(|F|, t)/|F| (Section 3.1 temperature cap)."""
    lib = _load()
    f = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
    D = np.zeros_like(f)
    _check(lib.orc_cap(f.size // 2, f, float(t), D), "cap")
    return D.reshape(-1, 2)


@dataclass
class StepStats:
    moved: int
    max_disp: float
    energy: float
    coincident: int


def step(n: int, row_ptr, col_idx, kptr, kidx, d: float, t: float, pos,
         stop_displacement: float = 0.01):
    """One synchronous iteration.  Returns (new_pos, F, Delta, StepStats)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1).copy()
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    F = np.zeros(2 * max(n, 1), dtype=np.float64)
    D = np.zeros(2 * max(n, 1), dtype=np.float64)
    st = _IterStats()
    _check(lib.orc_step(n, rp, ci, kp, ki, float(d), float(t), float(stop_displacement), p, F, D,
                        ctypes.byref(st)), "step")
    return (p.reshape(-1, 2), F[: 2 * n].reshape(-1, 2), D[: 2 * n].reshape(-1, 2),
            StepStats(int(st.moved), float(st.max_disp), float(st.energy), int(st.coincident)))


def layout(n: int, row_ptr, col_idx, kptr, kidx, d: float, temperature, pos,
           h0: int = 0, h_end: int | None = None, stop_fraction: float = 0.0,
           stop_displacement: float = 0.01):
    """Iterations h0 .. h_end-1.  Returns (pos, iterations_run, StepStats)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    temps = np.ascontiguousarray(temperature, dtype=np.float64)
    if h_end is None:
        h_end = temps.size
    if h_end > temps.size:
        raise ValueError("temperature schedule shorter than h_end")
    p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1).copy()
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    if temps.size == 0:
        temps = np.zeros(1)
    run = ctypes.c_int32(0)
    st = _IterStats()
    _check(lib.orc_layout(n, rp, ci, kp, ki, float(d), temps, int(h0), int(h_end),
                          float(stop_fraction), float(stop_displacement), p, ctypes.byref(run),
                          ctypes.byref(st)), "layout")
    return (p.reshape(-1, 2), int(run.value),
            StepStats(int(st.moved), float(st.max_disp), float(st.energy), int(st.coincident)))


def paper_schedule(n: float, aspect: float, d: float, iterations: int) -> np.ndarray:
    """sqrt((n/a) d) 0.93^h for h = 0..iterations-1 (Section 5.1)."""
    t = np.zeros(max(iterations, 1))
    _load().orc_paper_schedule(float(n), float(aspect), float(d), int(iterations), t)
    return t[:iterations]


def linear_schedule(t0: float, iterations: int) -> np.ndarray:
    """t0 - t0 h / iterations for h = 0..iterations-1."""
    t = np.zeros(max(iterations, 1))
    _load().orc_linear_schedule(float(t0), int(iterations), t)
    return t[:iterations]
