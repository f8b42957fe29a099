"""Summaries of rocprofv3 results (the SQLite databases it writes).

    python -m paper_1606_02162_amd.profsum trace DIR            # per-kernel stats
    python -m paper_1606_02162_amd.profsum counters DIR [KERNEL] # counter averages
    python -m paper_1606_02162_amd.profsum ranges DIR            # roctx ranges (--marker-trace)

and the traffic summary that bench.py reads:

    python -m paper_1606_02162_amd.profsum traffic --fetch DIR --write DIR \\
        --calib-fetch DIR --calib-write DIR --kernel NAME --out FILE.json

HBM traffic of a kernel is FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
scaled by bytes_known / counter_value of a plain device copy of known size
(bench.py --calibrate-copy copies 1 GiB three times).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys


def _db(path: str) -> str:
    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", "*results.db"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return hits[0]


def kernel_stats(path: str):
    """Per-kernel dispatch count, total and average duration (ns), share."""
    con = sqlite3.connect(_db(path))
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration) from kernels group by name "
                       "order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1.0
    return [{"name": r[0], "calls": r[1], "total_ns": r[2], "avg_ns": r[3], "min_ns": r[4],
             "max_ns": r[5], "pct": 100.0 * r[2] / total} for r in rows]


def counters(path: str, kernel: str | None = None, min_grid: int = 0, longest: bool = False):
    """Counter averages per kernel over its dispatches with at least min_grid
    threads; with `longest`, the values of each kernel's longest dispatch
    only (one launch among shorter ones of the same kernel)."""
    con = sqlite3.connect(_db(path))
    rows = con.execute("select kernel_name, counter_name, value, dispatch_id, duration, grid_size "
                       "from counters_collection").fetchall()
    picked = {}
    if longest:
        for name, _, _, did, dur, grid in rows:
            if grid >= min_grid and (name not in picked or dur > picked[name][1]):
                picked[name] = (did, dur)
    acc = {}
    for name, cname, val, did, dur, grid in rows:
        if kernel and kernel not in name:
            continue
        if grid < min_grid or (longest and picked[name][0] != did):
            continue
        a = acc.setdefault((name, cname), [0.0, 0, 0.0])
        a[0] += val
        a[1] += 1
        a[2] += dur
    out = []
    for (name, cname), (s, cnt, dur) in sorted(acc.items()):
        out.append({"kernel": name, "counter": cname, "avg": s / cnt, "dispatches": cnt,
                    "avg_duration_ns": dur / cnt})
    return out


def _one(path: str, kernel: str, counter: str, min_grid: int = 0, longest: bool = False) -> float:
    vals = [c["avg"] for c in counters(path, kernel, min_grid, longest) if c["counter"] == counter]
    if not vals:
        raise KeyError(f"{counter} for {kernel} not in {path}")
    return float(vals[0])


def traffic(fetch, write, calib_fetch, calib_write, kernel, calib_bytes=1 << 30, min_grid=0,
            longest=False):
    f = _one(fetch, kernel, "FETCH_SIZE", min_grid, longest)
    w = _one(write, kernel, "WRITE_SIZE", min_grid, longest)
    cf = _one(calib_fetch, "copyBuffer", "FETCH_SIZE")
    cw = _one(calib_write, "copyBuffer", "WRITE_SIZE")
    fs = calib_bytes / (cf * 1024.0)
    ws = calib_bytes / (cw * 1024.0)
    return {"kernel": kernel, "fetch_kib": f, "write_kib": w, "calib_fetch_kib": cf,
            "calib_write_kib": cw, "fetch_scale": fs, "write_scale": ws,
            "bytes_per_launch": f * 1024.0 * fs + w * 1024.0 * ws}


def source_hash(root: str, files) -> str:
    h = hashlib.sha256()
    for rel in files:
        with open(os.path.join(root, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def range_stats(path: str):
    """Per-name count, total, average and longest duration (ns) of the
    marker regions (roctx ranges and marks) of a --marker-trace run."""
    con = sqlite3.connect(_db(path))
    # the range's text is the message argument in the region's extdata
    rows = con.execute("select coalesce(json_extract(extdata, '$.message'), name) as label, "
                       "category, count(*), sum(duration), avg(duration), max(duration) "
                       "from regions where category like '%MARKER%' "
                       "group by label, category order by sum(duration) desc").fetchall()
    con.close()
    return [{"name": r[0], "category": r[1], "calls": r[2], "total_ns": r[3] or 0,
             "avg_ns": r[4] or 0, "max_ns": r[5] or 0} for r in rows]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--top", type=int, default=15)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("kernel", nargs="?")
    c.add_argument("--min-grid", type=int, default=0, help="only dispatches of >= this many threads")
    c.add_argument("--longest", action="store_true", help="only each kernel's longest dispatch")
    rg = sub.add_parser("ranges")
    rg.add_argument("dir")
    tr = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        tr.add_argument("--" + k.replace("_", "-"), required=True)
    tr.add_argument("--kernel", required=True)
    tr.add_argument("--min-grid", type=int, default=0)
    tr.add_argument("--longest", action="store_true")
    tr.add_argument("--out", required=True)
    tr.add_argument("--sources", nargs="*", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(f"{'kernel':<64} {'calls':>6} {'avg us':>10} {'min us':>9} {'max us':>9} "
              f"{'total ms':>10} {'%':>6}")
        for r in kernel_stats(a.dir)[: a.top]:
            print(f"{r['name'][:64]:<64} {r['calls']:>6} {r['avg_ns'] / 1e3:>10.1f} "
                  f"{r['min_ns'] / 1e3:>9.1f} {r['max_ns'] / 1e3:>9.1f} "
                  f"{r['total_ns'] / 1e6:>10.2f} {r['pct']:>6.2f}")
    elif a.cmd == "ranges":
        print(f"{'range':<48} {'calls':>7} {'avg ms':>10} {'max ms':>10} {'total ms':>11}")
        for r in range_stats(a.dir):
            print(f"{r['name'][:48]:<48} {r['calls']:>7} {r['avg_ns'] / 1e6:>10.3f} "
                  f"{r['max_ns'] / 1e6:>10.3f} {r['total_ns'] / 1e6:>11.2f}")
    elif a.cmd == "counters":
        for r in counters(a.dir, a.kernel, a.min_grid, a.longest):
            print(f"{r['kernel'][:60]:<60} {r['counter']:<28} {r['avg']:>16.6g} "
                  f"{r['dispatches']:>6}")
    else:
        res = traffic(a.fetch, a.write, a.calib_fetch, a.calib_write, a.kernel,
                      min_grid=a.min_grid, longest=a.longest)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if a.sources:
            res["source_files"] = a.sources
            res["source_sha256"] = source_hash(root, a.sources)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
