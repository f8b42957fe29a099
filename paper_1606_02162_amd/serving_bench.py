"""Serving benchmark: an open-loop Poisson stream of layout jobs through the
continuous-batching server, against the plain per-graph solver.

Jobs: Watts-Strogatz graphs (ring degree 6, rewiring probability 0.1) with n
log-uniform in [100, 200000], k uniform in {2, 3}, 200 iterations, initial
positions uniform in [0, 1200)^2, FP32 with Kahan-compensated sums.
Arrivals: exponential inter-arrival times at the given rate.  A submitter
thread submits each job at its arrival time; the latency of a job is from
its submission to its completion (measured by the server).  The baseline
runs the same jobs one after another through gila_layout (upload, build,
iterations, download) and replays the arrival times through that single
FIFO server to get its latencies.
"""
from __future__ import annotations

import json
import threading
import sys
import time

import numpy as np

from . import gila, inputs


# the server's default limit for small (batched) jobs
SMALL_MAX_N = 1024


def make_jobs(count: int, seed: int = 5):
    """The job list: graph, k and initial positions of each job.  Each job
    depends only on its index, so the jobs are generated on a thread pool
    (numpy's sorts release the interpreter lock)."""
    import concurrent.futures as cf
    import os
    sizes = inputs.log_uniform_sizes(count, 100, 200000, seed)
    rng = np.random.default_rng(seed)
    ks = rng.integers(2, 4, size=count)

    def one(i):
        g = inputs.watts_strogatz(int(sizes[i]), 6, 0.1, seed=5_000_000 + i)
        x0 = inputs.uniform_positions(g.n, seed=i, width=inputs.PAPER_FRAME)
        return (g, int(ks[i]), x0)

    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(count)))


def params_for(g, H=200):
    d = inputs.PAPER_IDEAL_LENGTH
    return gila.LayoutParams(temperature=gila.paper_schedule(g.n, 1.0, d, H), ideal_length=d,
                             precision=gila.FP32_KAHAN)


def run_server(jobs, arrivals, max_slots=256, config=None):
    srv = gila.Server(max_slots=max_slots)
    for key, value in (config or {}).items():
        srv.config(key, value)
    tickets = [None] * len(jobs)
    t0 = time.perf_counter()

    def submitter():
        for i, (g, k, x0) in enumerate(jobs):
            delay = arrivals[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[i] = srv.submit(g, k, params_for(g), x0)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    for t in tickets:
        srv.wait(t)
    t_end = time.perf_counter()
    lat = np.array([srv.latency(t)[1] for t in tickets])
    queued = np.array([srv.latency(t)[0] for t in tickets])
    info = srv.info()
    srv.close()
    return lat, queued, t_end - t0, info


def run_per_graph(jobs, sample):
    """Service time of each sampled job through the plain per-graph solver."""
    import torch
    svc = {}
    for i in sample:
        g, k, x0 = jobs[i]
        torch.cuda.synchronize()
        t = time.perf_counter()
        rp, ci = gila.to_device_csr(g)
        pos = torch.from_numpy(x0.astype(np.float32)).cuda()
        gila.layout(rp, ci, k, params_for(g), pos)
        _ = pos.cpu()
        svc[i] = time.perf_counter() - t
    return svc


def _progress(msg: str) -> None:
    print(f"[serve] {msg}", file=sys.stderr, flush=True)


def measure(args, job_records=None) -> dict:
    """The served form: the Poisson stream through the server, the same jobs
    through the per-graph solver as a FIFO queue.  Returns the result object
    (sub-config, throughput, latencies overall and by class, comparison);
    with a list as ``job_records``, appends one ``served_job`` record per job
    (its latency, interactions/s, algorithmic bytes/s, roofline fraction)."""
    import torch
    torch.cuda.set_device(0)
    count, rate = args.serve_jobs, args.serve_rate
    jobs = make_jobs(count)
    _progress(f"{count} jobs generated")
    arrivals = inputs.poisson_arrivals(count, rate, seed=5)
    arrivals = arrivals - arrivals[0]
    # warm-up: a few jobs (loads the kernels, fills the library's caches)
    warm = make_jobs(8, seed=99)
    run_server(warm, np.zeros(len(warm)))
    lat, queued, wall, info = run_server(jobs, arrivals)
    _progress(f"server run done in {wall:.1f} s")
    pairs, kpairs, actives = [], [], []
    for g, k, _ in jobs:
        # pairs per iteration counted by the library
        rp, ci = gila.to_device_csr(g)
        kh = gila.build_khop(rp, ci, k)
        inf = kh.info()
        pairs.append(inf["total_pairs"] + g.nnz)
        kpairs.append(inf["total_pairs"])
        actives.append(inf["n_active"])
        kh.free()
    if job_records is not None:
        from paper_1606_02162_amd import records
        for i, (g, k, _) in enumerate(jobs):
            job_records.append(records.job_record(
                lat[i] * 1e-3, kpairs[i], g.nnz, actives[i], 200, kind="served_job", job=i,
                n=g.n, k=k, queued_ms=float(queued[i]),
                note="submit to completion, host buffers in and out"))
    inter = float(np.sum(pairs)) * 200
    # plain per-graph solver on every 4th job; FIFO replay of the arrivals
    sample = list(range(0, count, 4))
    _progress("pairs counted; per-graph solver on every 4th job")
    svc = run_per_graph(jobs, sample)
    _progress("per-graph solver done")
    scale = float(np.sum([pairs[i] for i in range(count)])) / float(
        np.sum([pairs[i] for i in sample]))
    base_busy = sum(svc.values()) * scale
    # FIFO replay with each unsampled job's service time interpolated by pairs
    rate_pg = float(np.sum([pairs[i] for i in sample])) / sum(svc.values())
    service = np.array([svc.get(i, pairs[i] / rate_pg) for i in range(count)])
    finish, free_at = np.zeros(count), 0.0
    for i in range(count):
        start = max(arrivals[i], free_at)
        free_at = start + service[i]
        finish[i] = free_at
    base_lat = (finish - arrivals) * 1e3
    # latency by job class: small jobs go through batched LDS-resident launches
    small = np.array([g.n <= SMALL_MAX_N for g, _, _ in jobs])
    by_class = {}
    for name, mask in (("small", small), ("large", ~small)):
        if mask.any():
            by_class[name] = {"jobs": int(mask.sum()), "n_max": SMALL_MAX_N if name == "small"
                              else 200000,
                              "p50": float(np.percentile(lat[mask], 50)),
                              "p99": float(np.percentile(lat[mask], 99))}
    return {
        "config": {"workload": f"serve_ws_poisson{rate:g}_{count}jobs_k2or3_200iters",
                   "jobs": count, "warmup_jobs": len(warm), "rate_per_s": rate,
                   "n_range": [100, 200000], "k": [2, 3], "iterations": 200,
                   "precision": "f32 + Kahan",
                   "data": "synthetic: Watts-Strogatz ring degree 6, rewiring p = 0.1, n "
                           "log-uniform, Poisson arrivals, init uniform in [0,1200)^2"},
        "interactions_per_s": inter / wall,
        "wall_s": wall,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "queued_p50": float(np.percentile(queued, 50)),
                       "by_class": by_class},
        "server": info,
        "per_graph_solver": {
            "interactions_per_s": inter / base_busy,
            "latency_ms_fifo": {"p50": float(np.percentile(base_lat, 50)),
                                "p99": float(np.percentile(base_lat, 99))},
            "sampled_jobs": len(sample)},
    }


def main(args) -> int:
    jsonl = getattr(args, "jsonl", None)
    job_recs = [] if jsonl else None
    r = measure(args, job_recs)
    if jsonl:
        from paper_1606_02162_amd import records
        records.write_jsonl(jsonl, job_recs)
    out = {
        "metric": "served layouts: k-hop force interactions/s and p50/p99 latency",
        "value": r["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": r["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (Kahan lane sums)",
        "data": "synthetic", "config": r["config"], "latency_ms": r["latency_ms"],
        "server": r["server"], "per_graph_solver": r["per_graph_solver"],
    }
    print(json.dumps(out))
    return 0
