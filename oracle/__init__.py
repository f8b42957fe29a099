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
    ||f^r|| = d^2/delta^q (FR: p = 2, q = 1; the LinLog model of Section 6:
    p = 0, q = 1);
  * Section 4.5, the k-neighbourhood N_v(k), adjacent vertices receiving both
    forces, and the synchronous coordinate update;
  * Section 5.1, the cap schedule sqrt((n/a) d) 0.93^h and the halting rule;
  * Sections 4.3 and 4.6, pruning of degree-one vertices, repulsion weighted
    by the pruned leaves, and reinsertion of the leaves on a small circle;
  * Sections 4.6 and 5.1, connected components laid out one by one, each
    with the cap of its own vertex count and initial aspect ratio, and their
    drawings packed in a matrix;
  * Section 5.2, the drawing-quality metrics: crossings, edge length
    standard deviation, and the similarity of the drawing's Gabriel graph to
    the graph.
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
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    lib.orc_khop_count.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int32, ctypes.c_int64,
                                   vp, _i64p]
    lib.orc_khop_fill.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int32, ctypes.c_int64,
                                  vp, _i64p, _i32p]
    i32 = ctypes.c_int32
    lib.orc_forces.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int64, vp, _i64p, _i32p,
                               ctypes.c_double, vp, i32, i32, _f64p, _f64p,
                               ctypes.POINTER(ctypes.c_int64)]
    lib.orc_force_magnitudes.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int64, vp, _i64p,
                                         _i32p, ctypes.c_double, vp, i32, i32, _f64p, _f64p]
    lib.orc_cap.argtypes = [ctypes.c_int64, _f64p, ctypes.c_double, _f64p]
    lib.orc_step.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, ctypes.c_double, vp,
                             i32, i32, ctypes.c_double, ctypes.c_double, _f64p, _f64p, _f64p,
                             ctypes.POINTER(_IterStats)]
    lib.orc_layout.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, ctypes.c_double,
                               vp, i32, i32, _f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_double, _f64p, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(_IterStats)]
    lib.orc_paper_schedule.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, _f64p]
    lib.orc_linear_schedule.argtypes = [ctypes.c_double, ctypes.c_int32, _f64p]
    lib.orc_prune.argtypes = [ctypes.c_int32, _i64p, _i32p, _i32p, _i32p, _i32p,
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.orc_pruned_graph.argtypes = [ctypes.c_int32, _i64p, _i32p, _i32p, _i64p, _i32p]
    lib.orc_reinsert.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int32, _i64p,
                                 _i32p, ctypes.c_double, _f64p, _f64p]
    lib.orc_components.argtypes = [ctypes.c_int32, _i64p, _i32p, _i32p,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.orc_pack.argtypes = [ctypes.c_int32, _i32p, ctypes.c_double, _f64p]
    lib.orc_crossings.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, vp,
                                  ctypes.POINTER(ctypes.c_int64)]
    lib.orc_edge_crossings.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, ctypes.c_int64,
                                       _i64p, _i64p]
    lib.orc_edge_lengths.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.orc_gabriel.argtypes = [ctypes.c_int32, _f64p, _i64p, vp]
    lib.orc_jaccard.argtypes = [ctypes.c_int32, _i64p, _i32p, _i64p, _i32p, vp,
                                ctypes.POINTER(ctypes.c_double)]
    for f in ("orc_khop_count", "orc_khop_fill", "orc_forces", "orc_force_magnitudes", "orc_cap",
              "orc_step",
              "orc_layout", "orc_prune", "orc_pruned_graph", "orc_reinsert", "orc_components",
              "orc_pack", "orc_crossings", "orc_edge_crossings", "orc_edge_lengths", "orc_gabriel",
              "orc_jaccard"):
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


def _mass(mass, n):
    """(array, pointer) for an optional float64[n] weight vector (None = unit)."""
    if mass is None:
        return None, None
    arr = np.ascontiguousarray(mass, dtype=np.float64)
    if arr.size != n:
        raise ValueError("mass must hold one weight per vertex")
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _verts(verts):
    if verts is None:
        return None, None
    arr = np.ascontiguousarray(verts, dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not
    depend on it)."""
    lib = _load()
    lib.orc_set_threads.argtypes = [ctypes.c_int32]
    lib.orc_set_threads.restype = None
    lib.orc_set_threads(int(t))


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


def forces(n: int, row_ptr, col_idx, kptr, kidx, d: float, pos, verts=None, mass=None,
           p: int = 2, q: int = 1):
    """F_v for verts (Section 3.1 with N_v(k) repulsion, Section 4.5).

    ``kptr``/``kidx`` hold the rows of exactly the vertices in ``verts``
    (all vertices when verts is None).  ``pos`` is float64[n, 2].  ``mass``
    (float64[n], optional) scales the repulsion each vertex exerts
    (Section 4.6: 1 + its pruned leaves).  ``p``, ``q``: force exponents,
    ||f^a|| = delta^p / d and ||f^r|| = d^2 / delta^q (FR: 2, 1; LinLog: 0, 1).
    Returns (F float64[count, 2], coincident pair count).
    """
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    marr, mptr = _mass(mass, n)
    varr, vptr = _verts(verts)
    count = n if varr is None else varr.size
    pos_ = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    F = np.zeros(2 * max(count, 1), dtype=np.float64)
    coinc = ctypes.c_int64(0)
    _check(lib.orc_forces(n, rp, ci, count, vptr, kp, ki, float(d), mptr, int(p), int(q), pos_,
                          F, ctypes.byref(coinc)), "forces")
    return F[: 2 * count].reshape(count, 2), int(coinc.value)


def force_magnitudes(n: int, row_ptr, col_idx, kptr, kidx, d: float, pos, verts=None, mass=None,
                     p: int = 2, q: int = 1):
    """S_v = sum of the magnitudes of the terms of F_v (Section 3.1:
    delta^p / d per adjacent u, w_u d^2 / delta^q per u in N_v(k)); rows and
    arguments as in :func:`forces`.  Returns float64[count].

    S_v bounds |F_v|, and a force whose every term is rounded to a relative
    error e is off by at most e * S_v: the scale of a per-vertex gate.
    kappa_v = S_v / |F_v| is the condition number of the sum.
    """
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    marr, mptr = _mass(mass, n)
    varr, vptr = _verts(verts)
    count = n if varr is None else varr.size
    pos_ = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    S = np.zeros(max(count, 1), dtype=np.float64)
    _check(lib.orc_force_magnitudes(n, rp, ci, count, vptr, kp, ki, float(d), mptr, int(p),
                                    int(q), pos_, S), "force_magnitudes")
    return S[:count]


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
         stop_displacement: float = 0.01, mass=None, p: int = 2, q: int = 1):
    """One synchronous iteration.  Returns (new_pos, F, Delta, StepStats)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    marr, mptr = _mass(mass, n)
    x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1).copy()
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    F = np.zeros(2 * max(n, 1), dtype=np.float64)
    D = np.zeros(2 * max(n, 1), dtype=np.float64)
    st = _IterStats()
    _check(lib.orc_step(n, rp, ci, kp, ki, float(d), mptr, int(p), int(q), float(t),
                        float(stop_displacement), x, F, D, ctypes.byref(st)), "step")
    return (x.reshape(-1, 2), F[: 2 * n].reshape(-1, 2), D[: 2 * n].reshape(-1, 2),
            StepStats(int(st.moved), float(st.max_disp), float(st.energy), int(st.coincident)))


def layout(n: int, row_ptr, col_idx, kptr, kidx, d: float, temperature, pos,
           h0: int = 0, h_end: int | None = None, stop_fraction: float = 0.0,
           stop_displacement: float = 0.01, mass=None, p: int = 2, q: int = 1):
    """Iterations h0 .. h_end-1.  Returns (pos, iterations_run, StepStats)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    marr, mptr = _mass(mass, n)
    temps = np.ascontiguousarray(temperature, dtype=np.float64)
    if h_end is None:
        h_end = temps.size
    if h_end > temps.size:
        raise ValueError("temperature schedule shorter than h_end")
    x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1).copy()
    kp = np.ascontiguousarray(kptr, dtype=np.int64)
    ki = np.ascontiguousarray(kidx, dtype=np.int32)
    if ki.size == 0:
        ki = np.zeros(1, dtype=np.int32)
    if temps.size == 0:
        temps = np.zeros(1)
    run = ctypes.c_int32(0)
    st = _IterStats()
    _check(lib.orc_layout(n, rp, ci, kp, ki, float(d), mptr, int(p), int(q), temps, int(h0),
                          int(h_end), float(stop_fraction), float(stop_displacement), x,
                          ctypes.byref(run), ctypes.byref(st)), "layout")
    return (x.reshape(-1, 2), int(run.value),
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


@dataclass
class Pruned:
    """Result of pruning the degree-one vertices (Section 4.3).

    anchor[v]: the neighbour v was pruned from, -1 for kept vertices;
    leaves[v]: the number of vertices pruned from v;
    new_id[v]: v's id in the pruned graph (ascending original order), -1 if
    pruned; row_ptr/col_idx: the pruned graph; n: its vertex count.
    """
    anchor: np.ndarray
    leaves: np.ndarray
    new_id: np.ndarray
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray

    def mass(self) -> np.ndarray:
        """Weight of the repulsion exerted by each kept vertex (Section 4.6):
        1 + its pruned leaves, indexed by the pruned graph's ids."""
        kept = self.new_id >= 0
        m = np.zeros(self.n, dtype=np.float64)
        m[self.new_id[kept]] = 1.0 + self.leaves[kept]
        return m


def prune(n: int, row_ptr, col_idx) -> Pruned:
    """Remove the degree-one vertices (Section 4.3)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    anchor = np.zeros(max(n, 1), dtype=np.int32)
    leaves = np.zeros(max(n, 1), dtype=np.int32)
    new_id = np.zeros(max(n, 1), dtype=np.int32)
    nk = ctypes.c_int32(0)
    nnz = ctypes.c_int64(0)
    _check(lib.orc_prune(n, rp, ci, anchor, leaves, new_id, ctypes.byref(nk), ctypes.byref(nnz)),
           "prune")
    rpk = np.zeros(nk.value + 1, dtype=np.int64)
    cik = np.zeros(max(nnz.value, 1), dtype=np.int32)
    _check(lib.orc_pruned_graph(n, rp, ci, new_id, rpk, cik), "pruned_graph")
    return Pruned(anchor[:n], leaves[:n], new_id[:n], int(nk.value), rpk, cik[: nnz.value])


def reinsert(pr: Pruned, d: float, pos_kept) -> np.ndarray:
    """Place the pruned leaves around their neighbours (Section 4.6).

    pos_kept: float64[pr.n, 2], the pruned graph's drawing.  Returns
    float64[n, 2] for the original graph.
    """
    lib = _load()
    n = pr.anchor.size
    pk = np.ascontiguousarray(pos_kept, dtype=np.float64).reshape(-1)
    if pk.size != 2 * pr.n:
        raise ValueError("pos_kept must be [n_kept, 2]")
    if pk.size == 0:
        pk = np.zeros(2)
    out = np.zeros(2 * max(n, 1), dtype=np.float64)
    ci = pr.col_idx if pr.col_idx.size else np.zeros(1, dtype=np.int32)
    anchor = np.ascontiguousarray(pr.anchor if n else np.zeros(1, np.int32), dtype=np.int32)
    leaves = np.ascontiguousarray(pr.leaves if n else np.zeros(1, np.int32), dtype=np.int32)
    new_id = np.ascontiguousarray(pr.new_id if n else np.zeros(1, np.int32), dtype=np.int32)
    _check(lib.orc_reinsert(n, anchor, leaves, new_id, pr.n, pr.row_ptr, ci, float(d), pk, out),
           "reinsert")
    return out[: 2 * n].reshape(-1, 2)


def components(n: int, row_ptr, col_idx):
    """Connected components: (label int32[n] = smallest id of the component,
    count)."""
    lib = _load()
    rp, ci = _csr(row_ptr, col_idx)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    label = np.zeros(max(n, 1), dtype=np.int32)
    c = ctypes.c_int32(0)
    _check(lib.orc_components(n, rp, ci, label, ctypes.byref(c)), "components")
    return label[:n], int(c.value)


def pack(label, gap: float, pos) -> np.ndarray:
    """Components' drawings packed in a matrix (Section 4.6); returns new
    positions (float64[n, 2])."""
    lab = np.ascontiguousarray(label, dtype=np.int32)
    x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1).copy()
    n = lab.size
    if n == 0:
        return x.reshape(-1, 2)
    _check(_load().orc_pack(n, lab, float(gap), x), "pack")
    return x.reshape(-1, 2)


def component_aspect(x: np.ndarray) -> float:
    """Height / width of the frame enclosing a drawing (Section 5.1); 1 for a
    degenerate frame (zero width or height)."""
    w = float(x[:, 0].max() - x[:, 0].min())
    h = float(x[:, 1].max() - x[:, 1].min())
    return h / w if w > 0.0 and h > 0.0 else 1.0


def subgraph(row_ptr, col_idx, verts):
    """CSR of the subgraph induced by an ascending vertex list that is closed
    under adjacency (a union of components), in local ids (position in
    verts)."""
    rp, ci = _csr(row_ptr, col_idx)
    verts = np.asarray(verts, dtype=np.int64)
    local = np.full(rp.size - 1, -1, dtype=np.int64)
    local[verts] = np.arange(verts.size)
    lens = rp[verts + 1] - rp[verts]
    out_rp = np.zeros(verts.size + 1, dtype=np.int64)
    np.cumsum(lens, out=out_rp[1:])
    # entry j of the output is entry rp[v] + (j - out_rp[i]) of v's row
    first = np.repeat(rp[verts] - out_rp[:-1], lens)
    cols = local[ci[first + np.arange(out_rp[-1])]]
    if (cols < 0).any():
        raise ValueError("vertex list is not closed under adjacency")
    return out_rp, cols.astype(np.int32)


def layout_components(n: int, row_ptr, col_idx, k: int, d: float, iterations: int, pos,
                      stop_fraction: float = 0.15, stop_displacement: float = 0.01,
                      p: int = 2, q: int = 1, gap: float | None = None):
    """Sections 4.6 and 5.1: every connected component with at least two
    vertices is laid out on its own, from its vertices' positions in pos, with
    the cap sqrt((n_C / a_C) d) 0.93^h (n_C its vertex count, a_C the aspect
    ratio of its initial drawing) and its own halting rule; then the drawings
    are packed (gap d unless given).  Returns (pos, label, {label: iterations
    run})."""
    label, _ = components(n, row_ptr, col_idx)
    x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 2).copy()
    runs = {}
    # vertices grouped by label, ascending ids inside each group
    order = np.argsort(label, kind="stable")
    starts = np.flatnonzero(np.r_[True, label[order][1:] != label[order][:-1]]) if n else []
    bounds = list(starts) + [n]
    for j in range(len(bounds) - 1):
        verts = order[bounds[j]:bounds[j + 1]]
        root = label[verts[0]]
        if verts.size < 2:
            continue
        srp, sci = subgraph(row_ptr, col_idx, verts)
        x0 = x[verts]
        temps = paper_schedule(verts.size, component_aspect(x0), d, iterations)
        kp, ki = khop(verts.size, srp, sci, k)
        xf, run, _ = layout(verts.size, srp, sci, kp, ki, d, temps, x0,
                            stop_fraction=stop_fraction, stop_displacement=stop_displacement,
                            p=p, q=q)
        x[verts] = xf
        runs[int(root)] = run
    return pack(label, d if gap is None else gap, x), label, runs


def single(pos) -> np.ndarray:
    """A drawing at single precision (where the metrics are evaluated), as
    float64[n, 2]."""
    return np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 2)
                                .astype(np.float32).astype(np.float64))


def edge_list(row_ptr, col_idx):
    """Edges {u, v}, u < v, in row order: int32[m, 2]."""
    rp, ci = _csr(row_ptr, col_idx)
    v = np.repeat(np.arange(rp.size - 1, dtype=np.int32), np.diff(rp))
    keep = ci > v
    return np.stack([v[keep], ci[keep]], axis=1)


def crossings(n: int, row_ptr, col_idx, pos, per_edge: bool = False):
    """Number of crossing edge pairs of the drawing (Section 5.2), and with
    per_edge the crossings of every edge (edge_list order)."""
    rp, ci = _csr(row_ptr, col_idx)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    x = single(pos).reshape(-1)
    if x.size == 0:
        x = np.zeros(2)
    m = int(edge_list(row_ptr, col_idx).shape[0])
    pe = np.zeros(max(m, 1), dtype=np.int64)
    tot = ctypes.c_int64(0)
    _check(_load().orc_crossings(n, rp, ci, x, pe.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(tot)), "crossings")
    return (int(tot.value), pe[:m]) if per_edge else int(tot.value)


def edge_crossings(n: int, row_ptr, col_idx, pos, edges):
    """Crossings of the selected edges (indices into edge_list) with all edges."""
    rp, ci = _csr(row_ptr, col_idx)
    x = single(pos).reshape(-1)
    sel = np.ascontiguousarray(edges, dtype=np.int64)
    out = np.zeros(max(sel.size, 1), dtype=np.int64)
    _check(_load().orc_edge_crossings(n, rp, ci, x, sel.size, sel, out), "edge_crossings")
    return out[: sel.size]


def edge_lengths(n: int, row_ptr, col_idx, pos):
    """(mean, population standard deviation) of the edge lengths."""
    rp, ci = _csr(row_ptr, col_idx)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    x = single(pos).reshape(-1)
    if x.size == 0:
        x = np.zeros(2)
    mu, sd = ctypes.c_double(0), ctypes.c_double(0)
    _check(_load().orc_edge_lengths(n, rp, ci, x, ctypes.byref(mu), ctypes.byref(sd)),
           "edge_lengths")
    return float(mu.value), float(sd.value)


def gabriel(pos):
    """Gabriel graph of the drawing's points (brute force): (ptr, idx)."""
    x = single(pos)
    n = x.shape[0]
    xf = x.reshape(-1) if n else np.zeros(2)
    ptr = np.zeros(n + 1, dtype=np.int64)
    lib = _load()
    _check(lib.orc_gabriel(n, xf, ptr, None), "gabriel")
    idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
    _check(lib.orc_gabriel(n, xf, ptr, idx.ctypes.data_as(ctypes.c_void_p)), "gabriel")
    return ptr, idx[: int(ptr[-1])]


def similarity(n: int, row_ptr, col_idx, pos, per_vertex: bool = False):
    """Mean Jaccard index between each vertex's neighbourhood in the graph
    and in the drawing's Gabriel graph (Section 5.2)."""
    rp, ci = _csr(row_ptr, col_idx)
    gp, gi = gabriel(pos)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    if gi.size == 0:
        gi = np.zeros(1, dtype=np.int32)
    pv = np.zeros(max(n, 1))
    mean = ctypes.c_double(0)
    _check(_load().orc_jaccard(n, rp, ci, gp, gi, pv.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(mean)), "jaccard")
    return (float(mean.value), pv[:n]) if per_vertex else float(mean.value)
