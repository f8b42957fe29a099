"""JSON-lines records of layout runs: one JSON object per line, each with a
``kind`` -- ``iteration`` (the FP64 statistics of one iteration, as the
library's per-iteration history holds them, with the cap that iteration
used), ``job`` (one layout: latency, interactions/s, algorithmic bytes/s and
the fraction of the 8 TB/s HBM peak they are) or ``served_job`` (one job
through the layout server).  Plain Python: argument marshalling and file
output only."""
import json
import math

HBM_PEAK_BYTES_PER_S = 8.0e12


def algorithmic_bytes_per_iteration(pairs: int, nnz: int, n_active: int) -> int:
    """4 B per k-hop id and per adjacency entry, 32 B per active vertex (two
    row offsets, a position read and a position write)."""
    return 4 * int(pairs) + 4 * int(nnz) + 32 * int(n_active)


def iteration_records(history, temperature, h0: int = 0, **tags) -> list:
    """One record per row of ``history`` ((count, 4): energy, max
    displacement, moved, coincident, as ``KHop.history`` returns them), row j
    being iteration h0 + j; rows of iterations not run (NaN) are skipped."""
    out = []
    for j, row in enumerate(history):
        if any(math.isnan(float(x)) for x in row):
            continue
        h = h0 + j
        rec = {"kind": "iteration", "h": h, "cap": float(temperature[h]),
               "energy": float(row[0]), "max_disp": float(row[1]), "moved": int(row[2]),
               "coincident": int(row[3])}
        rec.update(tags)
        out.append(rec)
    return out


def job_record(latency_s: float, pairs: int, nnz: int, n_active: int, iterations: int,
               kind: str = "job", **tags) -> dict:
    """Latency, interactions/s ((P + 2m) per iteration), algorithmic bytes/s
    and their fraction of the HBM peak for one layout of ``iterations``
    iterations that took ``latency_s`` seconds."""
    inter = (int(pairs) + int(nnz)) * int(iterations)
    bps = algorithmic_bytes_per_iteration(pairs, nnz, n_active) * int(iterations) / latency_s
    rec = {"kind": kind, "latency_ms": latency_s * 1e3, "interactions": inter,
           "interactions_per_s": inter / latency_s, "bytes_per_s": bps,
           "roofline_frac": bps / HBM_PEAK_BYTES_PER_S}
    rec.update(tags)
    return rec


def write_jsonl(path: str, records, append: bool = False) -> int:
    """Writes the records, one per line; returns how many."""
    n = 0
    with open(path, "a" if append else "w") as f:
        for rec in records:
            f.write(json.dumps(rec, sort_keys=True) + "\n")
            n += 1
    return n


def read_jsonl(path: str) -> list:
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]
