"""Seeded synthetic inputs: graph generators and initial placements.

This module only *makes inputs*.  It contains none of the layout method's
arithmetic (no k-hop sets, no forces, no cooling); both the HIP library and
the CPU oracle receive what it produces as plain arrays.

Every graph is returned as a canonical simple undirected graph in symmetric
CSR form: ``row_ptr`` int64[n+1], ``col_idx`` int32[2m], rows sorted
ascending, no self-loops, no duplicate entries.  The paper removes isolated
vertices, self-loops and parallel edges from its real inputs (Section 5.2,
Table 1 caption); here self-loops and duplicates are removed and isolated
vertices are kept (they occur in R-MAT graphs).

Workload shapes follow the paper's benchmarks (Section 5.2): Erdos-Renyi
("Synth-Random") and Barabasi-Albert ("Synth-ScaleFree") graphs with density
m/n in [2, 3]; R-MAT stands in for the real co-purchasing network sizes of
Table 1 (amazon0302 has 262,111 vertices), and random trees plus extra edges
and Watts-Strogatz graphs shape the batched and served workloads.

Initial placement: the paper places vertices uniformly at random in a
1200 x 1200 frame (Section 5.1) without naming its generator.  Here the
uniform coordinates come from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a
counter-based generator, so that an independent implementation (the library's
device-side initialiser) can reproduce the exact same values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "to_csr", "grid_graph", "path_graph", "cycle_graph", "star_graph",
    "complete_graph", "erdos_renyi", "barabasi_albert", "rmat",
    "random_tree_plus_edges", "watts_strogatz", "splitmix64_u64",
    "splitmix64_uniform", "uniform_positions", "log_uniform_sizes",
    "poisson_arrivals", "PAPER_IDEAL_LENGTH", "PAPER_FRAME",
]

# d = N_s + sqrt(N_h^2 + N_w^2) with N_s = N_h = N_w = 20 (Section 5.1).
PAPER_IDEAL_LENGTH = 20.0 + math.sqrt(20.0 ** 2 + 20.0 ** 2)
# Side of the square frame of the random initial placement (Section 5.1).
PAPER_FRAME = 1200.0


@dataclass
class Graph:
    """A simple undirected graph in canonical symmetric CSR form."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[2m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self) -> np.ndarray:
        """Undirected edge list (u < v), shape [m, 2]."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def to_csr(n: int, u, v, name: str = "", meta: dict | None = None) -> Graph:
    """Canonicalise an edge list into a simple symmetric CSR graph.

    Self-loops are dropped, both directions are added, duplicates removed and
    every row sorted ascending.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * n + dst)
    src = key // n
    dst = key % n
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col_idx=dst.astype(np.int32), name=name,
                 meta=dict(meta or {}))


# --------------------------------------------------------------------------
# Deterministic small families (closed-form tests use these)
# --------------------------------------------------------------------------

def grid_graph(rows: int, cols: int) -> Graph:
    """rows x cols 4-neighbour grid; vertex id = cols * r + c."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    h_u, h_v = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    v_u, v_v = ids[:-1, :].ravel(), ids[1:, :].ravel()
    return to_csr(rows * cols, np.concatenate([h_u, v_u]), np.concatenate([h_v, v_v]),
                  name=f"grid{rows}x{cols}")


def path_graph(n: int) -> Graph:
    a = np.arange(n - 1)
    return to_csr(n, a, a + 1, name=f"path{n}")


def cycle_graph(n: int) -> Graph:
    a = np.arange(n)
    return to_csr(n, a, (a + 1) % n, name=f"cycle{n}")


def star_graph(leaves: int) -> Graph:
    """K_{1,leaves}: hub 0, leaves 1..leaves."""
    a = np.arange(1, leaves + 1)
    return to_csr(leaves + 1, np.zeros_like(a), a, name=f"star{leaves}")


def complete_graph(n: int) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    return to_csr(n, iu, ju, name=f"K{n}")


# --------------------------------------------------------------------------
# Random families (the paper's benchmark shapes)
# --------------------------------------------------------------------------

def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m): m distinct uniform edges without self-loops ("Synth-Random")."""
    rng = np.random.default_rng(seed)
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        ok = a != b
        lo = np.minimum(a, b)[ok]
        hi = np.maximum(a, b)[ok]
        cand = lo * n + hi
        # keep first occurrences, in draw order, of keys not seen yet
        _, first = np.unique(cand, return_index=True)
        cand = cand[np.sort(first)]
        cand = cand[~np.isin(cand, keys)]
        keys = np.concatenate([keys, cand[:need]])
    return to_csr(n, keys // n, keys % n, name=f"er{n}_{m}", meta={"seed": seed})


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Barabasi-Albert preferential attachment ("Synth-ScaleFree").

    The seed graph is a star on m+1 vertices (hub 0).  Every later vertex v
    attaches to m distinct earlier vertices, each drawn with probability
    proportional to its current degree (sampled from the list in which every
    vertex appears once per incident edge end).
    """
    if n <= m:
        raise ValueError("need n > m")
    rng = np.random.default_rng(seed)
    m_total = m + (n - m - 1) * m
    rep = np.empty(2 * m_total, dtype=np.int64)
    eu = np.empty(m_total, dtype=np.int64)
    ev = np.empty(m_total, dtype=np.int64)
    # seed star
    for i in range(1, m + 1):
        eu[i - 1], ev[i - 1] = 0, i
        rep[2 * (i - 1)], rep[2 * (i - 1) + 1] = 0, i
    ne = m
    length = 2 * m
    bulk = rng.random(8 * m * n + 64)
    bp = 0
    for v in range(m + 1, n):
        chosen: list[int] = []
        while len(chosen) < m:
            if bp >= bulk.size:
                bulk = rng.random(8 * m * n + 64)
                bp = 0
            t = int(rep[int(bulk[bp] * length)])
            bp += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            eu[ne], ev[ne] = v, t
            ne += 1
            rep[length], rep[length + 1] = v, t
            length += 2
    return to_csr(n, eu[:ne], ev[:ne], name=f"ba{n}_m{m}", meta={"seed": seed})


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = True) -> Graph:
    """R-MAT graph (Chakrabarti, Zhan and Faloutsos 2004), no noise.

    ``edge_factor * 2**scale`` directed pairs are drawn by recursive quadrant
    choice with probabilities a, b, c, d = 1-a-b-c; self-loops are dropped and
    the result symmetrised and deduplicated.  Unless ``permute`` is false the
    vertex ids are then relabelled by a seeded random permutation, so that id
    order carries no locality the generator did not create.  Isolated vertices
    are kept.
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    ne = edge_factor * n
    src = np.zeros(ne, dtype=np.int64)
    dst = np.zeros(ne, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for _ in range(scale):
        r = rng.random(ne)
        sbit = r >= ab
        dbit = ((r >= a) & (r < ab)) | (r >= abc)
        src = (src << 1) | sbit
        dst = (dst << 1) | dbit
    if permute:
        perm = rng.permutation(n)
        src, dst = perm[src], perm[dst]
    return to_csr(n, src, dst, name=f"rmat{scale}_ef{edge_factor}",
                  meta={"seed": seed, "a": a, "b": b, "c": c})


def random_tree_plus_edges(n: int, extra: int, seed: int) -> Graph:
    """Connected graph: random recursive tree plus ``extra`` random edges.

    Vertex i >= 1 attaches to a uniform j < i; then ``extra`` uniform edges
    that are neither loops nor duplicates are added.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(1, n, dtype=np.int64)
    parent = np.floor(rng.random(n - 1) * i).astype(np.int64)
    tu, tv = np.minimum(i, parent), np.maximum(i, parent)
    keys = tu * n + tv
    have = set(keys.tolist())
    extra = min(extra, n * (n - 1) // 2 - (n - 1))
    added: list[int] = []
    while len(added) < extra:
        need = extra - len(added)
        a = rng.integers(0, n, size=2 * need + 8)
        b = rng.integers(0, n, size=2 * need + 8)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y:
                continue
            kk = min(x, y) * n + max(x, y)
            if kk in have:
                continue
            have.add(kk)
            added.append(kk)
            if len(added) == extra:
                break
    allk = np.concatenate([keys, np.asarray(added, dtype=np.int64)])
    return to_csr(n, allk // n, allk % n, name=f"tree{n}+{extra}", meta={"seed": seed})


def watts_strogatz(n: int, degree: int, p: float, seed: int) -> Graph:
    """Watts-Strogatz small world: ring lattice, each edge rewired with prob. p.

    Each vertex u is joined to u+1 .. u+degree/2 (mod n).  Every lattice edge
    (u, u+j) is independently selected with probability p; a selected edge is
    replaced by (u, w) with w the first of four uniform draws that is neither
    u nor a lattice neighbour of u, and whose edge no earlier selected edge
    (in lattice order) has taken; if there is none the edge is kept.  The
    result is simple and keeps the lattice's edge count (all array work, so
    graphs of 10^5 vertices take milliseconds).
    """
    if degree % 2 or degree >= n:
        raise ValueError("degree must be even and < n")
    rng = np.random.default_rng(seed)
    half = degree // 2
    us = np.tile(np.arange(n, dtype=np.int64), half)
    js = np.repeat(np.arange(1, half + 1, dtype=np.int64), n)
    vs = (us + js) % n
    keys = np.minimum(us, vs) * n + np.maximum(us, vs)   # distinct, since degree < n
    sel = np.nonzero(rng.random(us.size) < p)[0]
    cand = rng.integers(0, n, size=(sel.size, 4))
    u_sel = us[sel][:, None]
    ckeys = np.minimum(u_sel, cand) * n + np.maximum(u_sel, cand)
    ring = np.abs(cand - u_sel)
    ok = np.minimum(ring, n - ring) > half   # neither u nor a lattice neighbour of u
    has = ok.any(axis=1)
    new = ckeys[np.arange(sel.size), ok.argmax(axis=1)]
    took = np.nonzero(has)[0]
    _, first = np.unique(new[took], return_index=True)   # first selected edge per new edge
    took = took[np.sort(first)]
    keys = keys.copy()
    keys[sel[took]] = new[took]
    return to_csr(n, keys // n, keys % n, name=f"ws{n}_k{degree}_p{p}",
                  meta={"seed": seed})


# --------------------------------------------------------------------------
# Counter-based uniform numbers and initial placements
# --------------------------------------------------------------------------

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_u64(seed: int, counters) -> np.ndarray:
    """Output number ``c`` (0-based) of a SplitMix64 stream seeded with ``seed``.

    state_c = seed + (c + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the
    SplitMix64 finaliser: z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.
    """
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, counters) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each output times 2^-53."""
    z = splitmix64_u64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_positions(n: int, seed: int, width: float = PAPER_FRAME,
                      height: float | None = None) -> np.ndarray:
    """float64[n, 2] uniform in [0, width) x [0, height).

    x_v uses counter 2v and y_v counter 2v+1 of the SplitMix64 stream; each
    coordinate is u * width (resp. u * height), rounded once to double.
    """
    if height is None:
        height = width
    c = np.arange(2 * n, dtype=np.uint64)
    u = splitmix64_uniform(seed, c).reshape(n, 2)
    out = np.empty((n, 2), dtype=np.float64)
    out[:, 0] = u[:, 0] * width
    out[:, 1] = u[:, 1] * height
    return out


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))) for ``count`` draws."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
