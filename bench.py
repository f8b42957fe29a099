"""Benchmark of the k-hop Fruchterman-Reingold layout on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one "step" = the whole hot path over one graph): build the k-hop
lists of an R-MAT graph with 2^18 vertices and edge factor 4 (a, b, c = 0.57,
0.19, 0.19; ~1.0M undirected edges after dedup), k = 2, then 500 layout
iterations in FP32 with Kahan-compensated force sums (FP64 reductions), paper
cap schedule, d = 20 + sqrt(800), initial placement uniform in [0, 1200)^2.
Inputs are generated and resident in HBM before timing starts.

Prints one JSON line.  value = (P + 2m) * H * steps / time, where P is the
total number of ordered k-hop pairs and 2m the adjacency entries (one force
term each per iteration).  The roofline object reports the force kernel's
achieved algorithmic bandwidth against the 8 TB/s HBM peak; cpu_baseline
times the FP64 CPU oracle on a bounded sample of the same job.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_seg_force_rmat18.json")
TRAFFIC_FILE_PRUNED = os.path.join(ROOT, "profiles", "traffic_seg_force_weighted_rmat18_pruned.json")
TRAFFIC_FILE_METRICS = os.path.join(ROOT, "profiles", "traffic_crossings_rmat18_layout.json")
TRAFFIC_FILE_BATCH = os.path.join(ROOT, "profiles", "traffic_batch_layout_batch4096.json")
TRAFFIC_FILE_BA = os.path.join(ROOT, "profiles", "traffic_seg_force_ba100k.json")
# counter summaries of the single-graph force kernels (FR model), by workload
TRAFFIC_FILE_BY_WORKLOAD = {"rmat": TRAFFIC_FILE, "ba": TRAFFIC_FILE_BA}
KERNEL_SOURCES = ["paper_1606_02162_amd/csrc/segment.hip", "paper_1606_02162_amd/csrc/iteration.h",
                  "paper_1606_02162_amd/csrc/gila_internal.h"]


def algorithmic_bytes_per_iter(P: int, nnz: int, n_active: int, pos_bytes: int = 8) -> int:
    """Compulsory HBM bytes of one iteration: 4 B per k-hop id, 4 B per
    adjacency id, and per non-isolated vertex its two row offsets (8 + 8 B),
    one position read and one position write (8 B each in FP32, 16 B in FP64)."""
    return 4 * P + 4 * nnz + (16 + 2 * pos_bytes) * n_active


def force_kernel_bytes(P: int, nnz: int, n_active: int, pos_bytes: int = 8) -> int:
    """The share of those bytes the force kernel moves: everything but the
    position write, which the combine kernel does."""
    return 4 * P + 4 * nnz + (16 + pos_bytes) * n_active


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path: str = TRAFFIC_FILE):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary, if it was taken on the kernel's sources (listed in the summary)
    as they are now."""
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("source_sha256") != kernel_source_hash(t.get("source_files") or KERNEL_SOURCES):
            return None
    except (OSError, ValueError):
        return None
    return t.get("bytes_per_launch")


def with_traffic_rate(obj):
    """Adds to every roofline object that carries measured HBM traffic the
    rate and fraction of peak that traffic gives at the kernel's measured
    duration ('achieved' and 'frac' are algorithmic-byte rates)."""
    if isinstance(obj, dict):
        r = obj.get("roofline")
        if isinstance(r, dict) and r.get("traffic") and r.get("kernel_ms") and r.get("unit") == "GB/s":
            rate = r["traffic"] / (r["kernel_ms"] * 1e-3) / 1e9
            r["traffic_GBps"] = rate
            r["traffic_frac"] = rate / r["peak"]
        for v in obj.values():
            with_traffic_rate(v)
    return obj


def single_graph_workloads(args):
    """The single-graph workloads: graph, k, iterations, precision, frame,
    ideal length and cap schedule of each."""
    from paper_1606_02162_amd import gila, inputs
    d = inputs.PAPER_IDEAL_LENGTH

    def paper_caps(g, H):
        n_active = int((np.diff(g.row_ptr) > 0).sum())
        return gila.paper_schedule(n_active, 1.0, d, H)

    return {
        # R-MAT scale 18, edge factor 4, k = 2, FP32 + Kahan, 500 iterations
        "rmat": dict(make=lambda: inputs.rmat(args.scale, 4, 0.57, 0.19, 0.19, seed=3), k=2,
                     H=args.iterations, precision=gila.FP32_KAHAN, frame=inputs.PAPER_FRAME,
                     d=d, caps=paper_caps, seed=0,
                     name=lambda H: f"rmat{args.scale}_ef4_k2_fp32kahan_{H}iters",
                     dtype="f32 (Kahan lane sums, f64 combine and reductions)",
                     metric="k-hop force interactions/s (P + 2m per iteration) at ~1M edges"),
        # Barabasi-Albert n = 100,000, m = 3, k = 3, FP32, [0, 1e4)^2, 300 iterations
        "ba": dict(make=lambda: inputs.barabasi_albert(100_000, 3, seed=2), k=3, H=300,
                   precision=gila.FP32, frame=1e4, d=d, caps=paper_caps, seed=0,
                   name=lambda H: f"ba100k_m3_k3_fp32_{H}iters", dtype="f32",
                   metric="k-hop force interactions/s (P + 2m per iteration), Barabasi-Albert 100k"),
        # 32 x 32 grid, k = 2, FP64, [0, 1000)^2, d = 10, cap 100 cooled linearly, 100 iterations
        "grid": dict(make=lambda: inputs.grid_graph(32, 32), k=2, H=100, precision=gila.FP64,
                     frame=1000.0, d=10.0, caps=lambda g, H: gila.linear_schedule(100.0, H),
                     seed=0, name=lambda H: f"grid32x32_k2_fp64_{H}iters", dtype="f64",
                     metric="k-hop force interactions/s (P + 2m per iteration), 32x32 grid"),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iterations", type=int, default=500, help="iterations of the rmat workload")
    ap.add_argument("--scale", type=int, default=18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--workload", choices=["rmat", "rmat_pruned", "rmat_components",
                                           "rmat_metrics", "ba", "grid", "batch", "serve"],
                    default="rmat",
                    help="rmat: one R-MAT graph (default line); rmat_pruned: the same graph "
                         "through pruning, leaf-weighted layout and reinsertion; ba: "
                         "Barabasi-Albert 100k; rmat_components: the same graph laid out "
                         "component by component with their own caps, then packed; "
                         "rmat_metrics: crossings, edge lengths and Gabriel similarity of its "
                         "layout; grid: "
                         "32x32 grid in FP64; batch: 4096 graphs "
                         "in one persistent launch; serve: Poisson stream through the layout "
                         "server")
    ap.add_argument("--model", default="fr",
                    help="force model of the single-graph workloads: fr (p = 2, q = 1), linlog "
                         "(p = 0, q = 1) or explicit exponents 'p,q'")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--per-graph-every", type=int, default=16,
                    help="the batched object times the plain per-graph solver on every N-th "
                         "graph, scaled by pair count")
    ap.add_argument("--no-batched", action="store_true",
                    help="default line without its batched (4096-graph) object")
    ap.add_argument("--no-served", action="store_true",
                    help="default line without its served (Poisson stream) object")
    ap.add_argument("--parity-samples", type=int, default=10000,
                    help="vertices sampled for the default line's parity object (0: none)")
    ap.add_argument("--jsonl", default=None, metavar="PATH",
                    help="also write JSON-lines records: every iteration's statistics of one "
                         "more run of the workload, one record for the timed layout, and one per "
                         "served job")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (three times) so that HBM "
                         "traffic counters can be scaled against a known byte count")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a large graph would "
              "be split by rows of its k-hop lists, balanced by pair count, with the positions "
              "all-gathered every iteration)", file=sys.stderr)
        return 2

    import torch

    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": x.numel() * 4,
                          "bytes_written": y.numel() * 4, "launches": 3}))
        return 0

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "rmat_pruned":
        return bench_pruned(args, single_graph_workloads(args)["rmat"])
    if args.workload == "rmat_components":
        return bench_components(args, single_graph_workloads(args)["rmat"])
    if args.workload == "rmat_metrics":
        return bench_metrics(args, single_graph_workloads(args)["rmat"])

    return bench_single(args, single_graph_workloads(args)[args.workload])


def force_model(args):
    """(library model id, p, q, name) of --model."""
    from paper_1606_02162_amd import gila
    m = args.model.strip().lower()
    if m == "fr":
        return gila.MODEL_FR, 2, 1, "fr"
    if m == "linlog":
        return gila.MODEL_LINLOG, 0, 1, "linlog"
    p, q = (int(x) for x in m.split(","))
    return gila.MODEL_PQ, p, q, f"p{p}q{q}"


def bench_single(args, wl) -> int:
    """One graph: a step is gila_build_khop + all iterations."""
    import torch

    from paper_1606_02162_amd import gila

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    g = wl["make"]()
    H, k, prec, d = wl["H"], wl["k"], wl["precision"], wl["d"]
    n_active = int((np.diff(g.row_ptr) > 0).sum())
    temps = wl["caps"](g, H)
    model, fp, fq, mname = force_model(args)
    params = gila.LayoutParams(temperature=temps, ideal_length=d, precision=prec,
                               force_model=model, force_p=fp, force_q=fq)
    rp, ci = gila.to_device_csr(g, dev)
    pos0 = torch.empty((g.n, 2), dtype=gila.position_dtype(prec), device=dev)
    gila.init_positions(g.n, wl["seed"], wl["frame"], wl["frame"], prec, pos0)
    pos = torch.empty_like(pos0)
    pos_bytes = 16 if prec == gila.FP64 else 8
    torch.cuda.synchronize()

    def one_step():
        pos.copy_(pos0)
        kh = gila.build_khop(rp, ci, k)
        st = gila.run(kh, params, pos)
        return kh, st

    for _ in range(args.warmup):
        kh, _ = one_step()
        kh.free()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    P = None
    for _ in range(args.steps):
        kh, st = one_step()
        if P is None:
            info = kh.info()
            P = info["total_pairs"]
        kh.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_s = t1 - t0
    assert st.iterations_run == H
    print(f"[bench] {args.steps} timed steps: {total_s * 1e3 / args.steps:.1f} ms each",
          file=sys.stderr, flush=True)

    # --- build time and iteration time, HIP events on the launch stream
    kh = gila.build_khop(rp, ci, k)
    pos.copy_(pos0)
    gila.run(kh, params, pos)    # a whole run first: the handle's memory and graph are warm
    pos.copy_(pos0)
    force_ms, combine_ms, timed_in_graph = gila.time_iterations(kh, params, pos, 0, min(50, H),
                                                                with_mode=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    pos.copy_(pos0)
    ev[0].record(stream)
    gila.run(kh, params, pos, 0, 0)            # reset + permute only
    ev[1].record(stream)
    ev[2].record(stream)
    gila.run(kh, params, pos)
    ev[3].record(stream)
    torch.cuda.synchronize()
    overhead_ms = ev[0].elapsed_time(ev[1])
    loop_ms = ev[2].elapsed_time(ev[3])
    iter_ms = max(loop_ms - overhead_ms, 1e-9) / H
    # build time as in the timed steps, where each build follows the free of
    # the previous handle and reuses its cached blocks: the first of three
    # builds allocates afresh (the timing handle above still holds memory)
    builds = []
    for _ in range(3):
        tb0 = time.perf_counter()
        kh2 = gila.build_khop(rp, ci, k)
        torch.cuda.synchronize()
        builds.append((time.perf_counter() - tb0) * 1e3)
        kh2.free()
    build_ms = min(builds[1:])

    copy_gbs = stream_copy_gbps(stream)
    inter_per_iter = P + g.nnz
    value = inter_per_iter * H * args.steps / total_s
    alg_bytes = algorithmic_bytes_per_iter(P, g.nnz, n_active, pos_bytes)
    kern_bytes = force_kernel_bytes(P, g.nnz, n_active, pos_bytes)
    achieved = kern_bytes / (force_ms * 1e-3) / 1e9
    prec_name = {gila.FP64: "FP64", gila.FP32: "FP32", gila.FP32_KAHAN: "FP32_KAHAN"}[prec]
    out = {
        "metric": wl["metric"],
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["dtype"],
        "data": "synthetic",
        "config": {"workload": wl["name"](H) + ("" if mname == "fr" else "_" + mname),
                   "n": g.n, "m": g.m, "k": k, "iterations": H, "total_pairs": P,
                   "n_active": n_active, "force_model": {"p": fp, "q": fq}},
        "ms_per_iter": iter_ms,
        "build_ms": build_ms,
        "build_ms_fresh_memory": builds[0],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(TRAFFIC_FILE_BY_WORKLOAD[args.workload])
                                 if mname == "fr" and args.workload in TRAFFIC_FILE_BY_WORKLOAD
                                 else None),
                     "kernel": f"seg_force_kernel<{prec_name}" + (">" if fq == 1 else ", q>") +
                               ("" if mname == "fr" else f" ({mname})"),
                     "kernel_ms": force_ms,
                     "algorithmic_bytes_per_launch": kern_bytes,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "iteration": {"ms": iter_ms, "force_kernel_ms": force_ms,
                      "combine_and_stats_ms": combine_ms,
                      "kernel_timing": ("one replay of 50 captured iterations between HIP "
                                        f"events ({force_ms + combine_ms:.4f} ms each); the "
                                        "force kernel's span from its first workgroup's start "
                                        "to its last one's end on the device wall clock; "
                                        "rest = iteration - force"
                                        + ("" if timed_in_graph else " (eager launches)")),
                      "algorithmic_bytes": alg_bytes,
                      "achieved_GBps": alg_bytes / (iter_ms * 1e-3) / 1e9},
    }

    if not args.no_cpu_baseline:
        # the oracle leg: the only place the benchmark calls the oracle
        import oracle
        threads = oracle.num_threads()
        if args.workload == "rmat" and mname == "fr" and args.parity_samples > 0:
            print("[bench] parity against the oracle", file=sys.stderr, flush=True)
            out["parity"] = parity_leg(args, g, k, d, temps, kh, pos0, oracle)
        print("[bench] oracle baseline", file=sys.stderr, flush=True)
        tc0 = time.perf_counter()
        optr, oidx = oracle.khop(g.n, g.row_ptr, g.col_idx, k)
        tc1 = time.perf_counter()
        x = pos0.double().cpu().numpy()
        for h in range(args.cpu_iters):
            x, _, _, _ = oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, d, temps[h], x,
                                     p=fp, q=fq)
        tc2 = time.perf_counter()
        cpu_build, cpu_iter = tc1 - tc0, (tc2 - tc1) / args.cpu_iters
        cpu_job = cpu_build + H * cpu_iter
        # one iteration on a single core, for the per-core figure
        oracle.set_threads(1)
        ts0 = time.perf_counter()
        oracle.step(g.n, g.row_ptr, g.col_idx, optr, oidx, d, temps[0], pos0.double().cpu().numpy(),
                    p=fp, q=fq)
        single_iter = time.perf_counter() - ts0
        oracle.set_threads(threads)
        out["cpu_baseline"] = {
            "value": inter_per_iter * H / cpu_job, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle on this host ({_cpu_model()}, {threads} threads): k-hop "
                       f"build once ({cpu_build:.2f} s) + {args.cpu_iters} iterations "
                       f"({cpu_iter * 1e3:.0f} ms each) of the same graph, extrapolated to "
                       f"the {H}-iteration job; single core: one iteration in "
                       f"{single_iter * 1e3:.0f} ms"),
            "single_core_iteration_value": inter_per_iter / single_iter,
        }
    if args.jsonl:
        from paper_1606_02162_amd import records
        kh.enable_history(H)
        pos.copy_(pos0)
        gila.run(kh, params, pos)
        recs = records.iteration_records(kh.history(), temps, workload=out["config"]["workload"])
        recs.append(records.job_record(total_s / args.steps, P, g.nnz, n_active, H,
                                       workload=out["config"]["workload"],
                                       note="one timed step: k-hop build + all iterations"))
        records.write_jsonl(args.jsonl, recs)
        kh.enable_history(0)
    kh.free()
    if args.workload == "rmat" and mname == "fr":
        if not args.no_batched:
            print("[bench] batched form", file=sys.stderr, flush=True)
            out["batched"] = batched_leg(args, args.steps, args.warmup)
        if not args.no_served:
            print("[bench] served form", file=sys.stderr, flush=True)
            from paper_1606_02162_amd import serving_bench
            job_recs = [] if args.jsonl else None
            out["served"] = serving_bench.measure(args, job_recs)
            if args.jsonl:
                from paper_1606_02162_amd import records
                records.write_jsonl(args.jsonl, job_recs, append=True)
    print(json.dumps(with_traffic_rate(out)))
    return 0


def parity_leg(args, g, k, d, temps, kh, pos0, oracle) -> dict:
    """Per-step error of the benchmark's GPU trajectory against the FP64 oracle
    (part of the oracle leg).  The GPU runs the benchmark's iterations; at
    h in {0, H/10, H/4, H/2, 3H/4, H-1} one step is taken with its force and
    displacement outputs, and the oracle recomputes that step from the same
    positions for a sample of non-isolated vertices (uniform, plus the 16
    largest degrees): F_v, S_v (sum of the term magnitudes), Delta_v
    (Section 3.1 cap) and x_v + Delta_v.  Reported per checkpoint:
    e_F = ||F_gpu - F_orc|| / ||F_orc|| and e_D (the same for Delta) over the
    sample, e_x = max |x_gpu - x_orc| / extent of the step's output
    positions, max_v |F_gpu - F_orc| / S_v, and kappa_v = S_v / |F_orc,v|
    (p50 / p99 / max).  Plain FP32 is run beside FP32 + Kahan."""
    import torch

    from paper_1606_02162_amd import gila

    H = len(temps)
    checks = sorted({0, H // 10, H // 4, H // 2, 3 * H // 4, H - 1})
    deg = np.diff(g.row_ptr)
    active = np.nonzero(deg > 0)[0]
    rng = np.random.default_rng(17)
    take = min(args.parity_samples, active.size)
    sample = np.unique(np.concatenate([rng.choice(active, take, replace=False),
                                       np.argsort(-deg)[:16]])).astype(np.int32)
    t0 = time.perf_counter()
    sp, si = oracle.khop(g.n, g.row_ptr, g.col_idx, k, verts=sample)
    res = {"config": "the benchmark graph and schedule (R-MAT 18, k = 2, 500 iterations), "
                     "initial positions as timed",
           "sample_vertices": int(sample.size), "sample_pairs": int(sp[-1]),
           "checkpoints": checks, "gates": {"e_F": 1e-5, "e_x": 1e-5}}
    for name, prec in (("fp32_kahan", gila.FP32_KAHAN), ("fp32", gila.FP32)):
        params = gila.LayoutParams(temperature=temps, ideal_length=d, precision=prec)
        pos = pos0.clone()
        F = torch.zeros((g.n, 2), dtype=torch.float64, device=pos.device)
        D = torch.zeros_like(F)
        done, rows = 0, {}
        for h in checks:
            if h > done:
                gila.run(kh, params, pos, done, h)
            x = pos.double().cpu().numpy()
            gila.step(kh, params, h, pos, F, D)
            xn = pos.double().cpu().numpy()
            done = h + 1
            Fg, Dg = F.cpu().numpy()[sample], D.cpu().numpy()[sample]
            Fo, _ = oracle.forces(g.n, g.row_ptr, g.col_idx, sp, si, d, x, verts=sample)
            So = oracle.force_magnitudes(g.n, g.row_ptr, g.col_idx, sp, si, d, x, verts=sample)
            Do = oracle.cap(Fo, float(temps[h]))
            xo = x[sample] + Do
            ext = max(float(np.ptp(xn[:, 0])), float(np.ptp(xn[:, 1])))
            nF = np.hypot(Fo[:, 0], Fo[:, 1])
            live = nF > 0
            kappa = So[live] / nF[live]
            dF = np.hypot(Fg[:, 0] - Fo[:, 0], Fg[:, 1] - Fo[:, 1])
            rows[str(h)] = {
                "e_F": float(np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo)),
                "e_x": float(np.hypot(*(xn[sample] - xo).T).max() / ext),
                "e_D": float(np.linalg.norm(Dg - Do) / max(np.linalg.norm(Do), 1e-300)),
                "max_dF_over_S": float((dF[So > 0] / So[So > 0]).max()),
                "kappa": {"p50": float(np.percentile(kappa, 50)),
                          "p99": float(np.percentile(kappa, 99)), "max": float(kappa.max())},
                "cap": float(temps[h])}
        worst = {key: max(r[key] for r in rows.values()) for key in ("e_F", "e_x", "e_D",
                                                                    "max_dF_over_S")}
        res[name] = {"steps": rows, "worst": worst,
                     "gates_met": worst["e_F"] <= 1e-5 and worst["e_x"] <= 1e-5}
    res["oracle_s"] = time.perf_counter() - t0
    return res


def bench_pruned(args, wl) -> int:
    """The R-MAT workload through the pipeline of Sections 4.3 - 4.6: a step
    is prune + k-hop build of the pruned graph + leaf weights + all
    iterations (captured loop) + reinsertion."""
    import torch

    from paper_1606_02162_amd import gila

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    g = wl["make"]()
    H, k, prec, d = wl["H"], wl["k"], wl["precision"], wl["d"]
    rp, ci = gila.to_device_csr(g, dev)
    pos0 = torch.empty((g.n, 2), dtype=gila.position_dtype(prec), device=dev)
    gila.init_positions(g.n, wl["seed"], wl["frame"], wl["frame"], prec, pos0)
    pos = torch.empty_like(pos0)
    pos_bytes = 16 if prec == gila.FP64 else 8

    P0 = gila.prune(rp, ci)
    pinfo = P0.info()
    csr0, _ = P0.graph()
    g_pr = {"n": csr0.n, "nnz": csr0.nnz}
    kh0 = gila.KHop.from_csr(csr0, k)
    kinfo = kh0.info()
    kh0.free()
    n_active = kinfo["n_active"]
    temps = gila.paper_schedule(n_active, 1.0, d, H)
    model, fp, fq, mname = force_model(args)
    params = gila.LayoutParams(temperature=temps, ideal_length=d, precision=prec,
                               force_model=model, force_p=fp, force_q=fq)
    kept = torch.empty((pinfo["n_kept"], 2), dtype=pos0.dtype, device=dev)
    torch.cuda.synchronize()

    def one_step():
        pos.copy_(pos0)
        Pr = gila.prune(rp, ci)
        csr, mass = Pr.graph()
        kh = gila.KHop.from_csr(csr, k)
        kh.set_mass(mass)
        Pr.gather(prec, pos, kept)
        st = gila.run(kh, params, kept)
        Pr.reinsert(d, prec, kept, pos)
        return Pr, kh, st

    for _ in range(args.warmup):
        Pr, kh, _ = one_step()
        kh.free()
        Pr.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Pr, kh, st = one_step()
        kh.free()
        Pr.free()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    assert st.iterations_run == H

    # phases: pruning, reinsertion, weighted and unweighted force kernels
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    Pr = gila.prune(rp, ci)
    ev[1].record(stream)
    torch.cuda.synchronize()
    prune_ms = ev[0].elapsed_time(ev[1])
    csr, mass = Pr.graph()
    kh = gila.KHop.from_csr(csr, k)
    Pr.gather(prec, pos0, kept)
    gila.time_iterations(kh, params, kept, 0, min(50, H))     # warm handle
    Pr.gather(prec, pos0, kept)
    plain_ms, _ = gila.time_iterations(kh, params, kept, 0, min(50, H))
    kh.set_mass(mass)
    Pr.gather(prec, pos0, kept)
    gila.time_iterations(kh, params, kept, 0, min(50, H))     # warm weighted layout
    Pr.gather(prec, pos0, kept)
    force_ms, combine_ms = gila.time_iterations(kh, params, kept, 0, min(50, H))
    ev[2].record(stream)
    Pr.reinsert(d, prec, kept, pos)
    ev[3].record(stream)
    torch.cuda.synchronize()
    reinsert_ms = ev[2].elapsed_time(ev[3])
    P = kinfo["total_pairs"]
    nnz = g_pr["nnz"]
    inter_per_iter = P + nnz
    value = inter_per_iter * H * args.steps / total_s
    # the weighted kernel also reads one FP32 weight per staged vertex
    w_bytes = 4 if prec != gila.FP64 else 8
    kern_bytes = force_kernel_bytes(P, nnz, n_active, pos_bytes) + w_bytes * n_active
    achieved = kern_bytes / (force_ms * 1e-3) / 1e9
    prec_name = {gila.FP64: "FP64", gila.FP32: "FP32", gila.FP32_KAHAN: "FP32_KAHAN"}[prec]
    out = {
        "metric": "k-hop force interactions/s of the pruned graph (P + 2m per iteration), "
                  "prune + weighted layout + reinsertion",
        "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"],
        "data": "synthetic",
        "config": {"workload": (wl["name"](H).replace("rmat", "rmat_pruned", 1) +
                                ("" if mname == "fr" else "_" + mname)), "n": g.n,
                   "m": g.m, "k": k, "iterations": H, "n_kept": pinfo["n_kept"],
                   "n_pruned": pinfo["n_pruned"], "m_kept": nnz // 2, "total_pairs": P,
                   "n_active": n_active, "force_model": {"p": fp, "q": fq}},
        "prune_ms": prune_ms, "reinsert_ms": reinsert_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(TRAFFIC_FILE_PRUNED) if mname == "fr" else None,
                     "kernel": f"seg_force_kernel<{prec_name}, weighted>", "kernel_ms": force_ms,
                     "algorithmic_bytes_per_launch": kern_bytes},
        "unweighted_force_kernel_ms": plain_ms,
        "combine_kernel_ms": combine_ms,
    }
    kh.free()
    Pr.free()

    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.num_threads()
        tc0 = time.perf_counter()
        pr = oracle.prune(g.n, g.row_ptr, g.col_idx)
        optr, oidx = oracle.khop(pr.n, pr.row_ptr, pr.col_idx, k)
        tc1 = time.perf_counter()
        x = pos0.double().cpu().numpy()[pr.new_id >= 0]
        m = pr.mass()
        for h in range(args.cpu_iters):
            x, _, _, _ = oracle.step(pr.n, pr.row_ptr, pr.col_idx, optr, oidx, d, temps[h], x,
                                     mass=m, p=fp, q=fq)
        tc2 = time.perf_counter()
        oracle.reinsert(pr, d, x)
        tc3 = time.perf_counter()
        cpu_build, cpu_iter = tc1 - tc0, (tc2 - tc1) / args.cpu_iters
        cpu_job = cpu_build + H * cpu_iter + (tc3 - tc2)
        out["cpu_baseline"] = {
            "value": inter_per_iter * H / cpu_job, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle on this host ({_cpu_model()}, {threads} threads): prune + "
                       f"k-hop build ({cpu_build:.2f} s), {args.cpu_iters} weighted iterations "
                       f"({cpu_iter * 1e3:.0f} ms each) extrapolated to {H}, reinsertion "
                       f"({(tc3 - tc2) * 1e3:.0f} ms)"),
        }
    print(json.dumps(with_traffic_rate(out)))
    return 0


def bench_components(args, wl) -> int:
    """The R-MAT workload through the per-component pipeline of Sections 4.6
    and 5.1: a step is gila_layout_components (labels, component order, every
    component of two or more vertices with its own cap -- the giant one on
    the whole GPU, the small ones in one batched launch -- and packing).  The
    halting rule is off so that every component runs all iterations."""
    import torch

    from paper_1606_02162_amd import gila

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    g = wl["make"]()
    H, k, prec, d = wl["H"], wl["k"], wl["precision"], wl["d"]
    n_active = int((np.diff(g.row_ptr) > 0).sum())
    model, fp, fq, mname = force_model(args)
    params = gila.LayoutParams(temperature=np.zeros(H), ideal_length=d, precision=prec,
                               force_model=model, force_p=fp, force_q=fq)
    rp, ci = gila.to_device_csr(g, dev)
    pos0 = torch.empty((g.n, 2), dtype=gila.position_dtype(prec), device=dev)
    gila.init_positions(g.n, wl["seed"], wl["frame"], wl["frame"], prec, pos0)
    pos = torch.empty_like(pos0)
    pos_bytes = 16 if prec == gila.FP64 else 8
    torch.cuda.synchronize()

    def one_step():
        pos.copy_(pos0)
        return gila.layout_components(rp, ci, k, params, pos)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, its = one_step()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    assert int(its.max()) == H

    # phases: labels, packing; the force kernel on the graph's lists (the giant
    # component holds nearly every row)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    label, _ = gila.components(rp, ci)
    ev[1].record(stream)
    ev[2].record(stream)
    gila.pack_components(label, d, prec, pos)
    ev[3].record(stream)
    torch.cuda.synchronize()
    label_ms, pack_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    kh = gila.build_khop(rp, ci, k)
    P = kh.info()["total_pairs"]
    tparams = gila.LayoutParams(temperature=gila.paper_schedule(n_active, 1.0, d, H),
                                ideal_length=d, precision=prec, force_model=model, force_p=fp,
                                force_q=fq)
    pos.copy_(pos0)
    gila.time_iterations(kh, tparams, pos, 0, min(50, H))      # warm handle
    pos.copy_(pos0)
    force_ms, _ = gila.time_iterations(kh, tparams, pos, 0, min(50, H))
    kh.free()
    inter_per_iter = P + g.nnz
    value = inter_per_iter * H * args.steps / total_s
    kern_bytes = force_kernel_bytes(P, g.nnz, n_active, pos_bytes)
    achieved = kern_bytes / (force_ms * 1e-3) / 1e9
    prec_name = {gila.FP64: "FP64", gila.FP32: "FP32", gila.FP32_KAHAN: "FP32_KAHAN"}[prec]
    sizes = np.bincount(label.cpu().numpy())
    sizes = sizes[sizes > 0]
    out = {
        "metric": "k-hop force interactions/s (P + 2m per iteration), every component laid out "
                  "with its own cap, then packed",
        "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"],
        "data": "synthetic",
        "config": {"workload": (wl["name"](H).replace("rmat", "rmat_components", 1) +
                                ("" if mname == "fr" else "_" + mname)), "n": g.n, "m": g.m,
                   "k": k, "iterations": H, "components": int(C),
                   "largest_component": int(sizes.max()),
                   "components_2_or_more": int((sizes >= 2).sum()), "total_pairs": P,
                   "force_model": {"p": fp, "q": fq}},
        "labels_ms": label_ms, "pack_ms": pack_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"seg_force_kernel<{prec_name}> (the graph's k-hop lists)",
                     "kernel_ms": force_ms, "algorithmic_bytes_per_launch": kern_bytes},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.num_threads()
        x0 = pos0.double().cpu().numpy()
        tc0 = time.perf_counter()
        oracle.layout_components(g.n, g.row_ptr, g.col_idx, k, d, 1, x0, stop_fraction=0.0,
                                 p=fp, q=fq)
        tc1 = time.perf_counter()
        oracle.layout_components(g.n, g.row_ptr, g.col_idx, k, d, 1 + args.cpu_iters, x0,
                                 stop_fraction=0.0, p=fp, q=fq)
        tc2 = time.perf_counter()
        cpu_iter = ((tc2 - tc1) - (tc1 - tc0)) / args.cpu_iters
        cpu_job = (tc1 - tc0) + (H - 1) * cpu_iter
        out["cpu_baseline"] = {
            "value": inter_per_iter * H / cpu_job, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle on this host ({_cpu_model()}, {threads} threads): the "
                       f"per-component pipeline with 1 and {1 + args.cpu_iters} iterations "
                       f"({tc1 - tc0:.2f} s, {tc2 - tc1:.2f} s); the difference gives "
                       f"{cpu_iter * 1e3:.0f} ms per iteration, extrapolated to {H}"),
        }
    print(json.dumps(with_traffic_rate(out)))
    return 0


# VALU lane operations per edge pair of the crossing test: four filtered
# orientation signs (multiply, fused multiply-add, add and a bound compare
# each) and two sign products with their compares; the combination of the
# lane masks runs on the scalar unit
CROSS_VALU_PER_PAIR = 20
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9  # CUs x lanes per cycle x clock


def bench_metrics(args, wl) -> int:
    """The drawing-quality metrics of Section 5.2 on the R-MAT 18 layout
    (build + 500 iterations, untimed): a step is one gila_drawing_metrics
    call with all three metrics (totals; no per-edge or per-vertex arrays).
    value = m(m-1)/2 edge pairs tested per second."""
    import torch

    from paper_1606_02162_amd import gila

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    g = wl["make"]()
    H, k, prec, d = wl["H"], wl["k"], wl["precision"], wl["d"]
    rp, ci = gila.to_device_csr(g, dev)
    pos = torch.empty((g.n, 2), dtype=gila.position_dtype(prec), device=dev)
    gila.init_positions(g.n, wl["seed"], wl["frame"], wl["frame"], prec, pos)
    params = gila.LayoutParams(temperature=wl["caps"](g, H), ideal_length=d, precision=prec)
    kh = gila.build_khop(rp, ci, k)
    gila.run(kh, params, pos)
    kh.free()
    m = g.m
    for _ in range(args.warmup):
        gila.drawing_metrics(rp, ci, prec, pos, 7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        met = gila.drawing_metrics(rp, ci, prec, pos, 7)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    part = {}
    for name, flag in (("crossings", gila.METRIC_CROSSINGS), ("lengths", gila.METRIC_LENGTHS),
                       ("similarity", gila.METRIC_SIMILARITY)):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        gila.drawing_metrics(rp, ci, prec, pos, flag)
        ev[1].record(stream)
        torch.cuda.synchronize()
        part[name] = ev[0].elapsed_time(ev[1])
    pairs = float(m) * float(m - 1) / 2.0
    value = pairs * args.steps / total_s
    cross_rate = pairs / (part["crossings"] * 1e-3)
    peak_rate = VALU_LANE_OPS_PER_S / CROSS_VALU_PER_PAIR
    out = {
        "metric": "edge pairs tested for crossings per second, with edge length deviation and "
                  "Gabriel similarity, on the R-MAT 18 layout",
        "value": value, "unit": "edge pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 coordinates, exact f64 signs; f64 sums", "data": "synthetic",
        "config": {"workload": "rmat_metrics18_ef4_k2_fp32kahan_500iters_layout", "n": g.n, "m": m},
        "metrics": dict(met.as_dict(), crossings_per_edge=met.crossings_per_edge),
        "ms": part,
        "roofline": {"bound": "alu", "achieved": cross_rate / 1e9, "peak": peak_rate / 1e9,
                     "unit": "Gpairs/s", "frac": cross_rate / peak_rate,
                     "traffic": measured_traffic(TRAFFIC_FILE_METRICS),
                     "kernel": "crossings_kernel", "kernel_ms": part["crossings"],
                     "valu_per_pair": CROSS_VALU_PER_PAIR},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.num_threads()
        x = pos.double().cpu().numpy()
        ns = 1536
        sel = np.random.default_rng(1).choice(m, ns, replace=False)
        tc0 = time.perf_counter()
        oracle.edge_crossings(g.n, g.row_ptr, g.col_idx, x, sel)
        tc1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": float(ns) * m / (tc1 - tc0), "unit": "edge pairs/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"exact-sign oracle on this host ({_cpu_model()}, {threads} threads): the "
                       f"crossings of {ns} sampled edges with all {m} edges ({tc1 - tc0:.2f} s); "
                       f"the oracle's Gabriel graph is cubic and not timed at this size"),
        }
    print(json.dumps(with_traffic_rate(out)))
    return 0


def stream_copy_gbps(stream) -> float:
    """Bytes read + written per second by a plain 1 GiB device copy (best of
    three, HIP events): the measured streaming ceiling beside the 8 TB/s
    specification."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        y.copy_(x)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def _percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return None, None
    return float(np.percentile(x, 50)), float(np.percentile(x, 99))


def batched_leg(args, steps: int, warmup: int) -> dict:
    """Many graphs in one persistent launch: 4096 connected graphs (random
    recursive tree + 0.5n extra edges, n log-uniform in [50, 5000]), k = 3,
    FP32, 200 iterations each.  A step is the k-hop build + the captured
    launch over the whole batch.  The same graphs through the plain per-graph
    solver (gila_layout one after another) are timed on every 16th graph
    (--per-graph-every) and scaled by pair count."""
    import torch

    from paper_1606_02162_amd import gila, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    count, H, k = args.batch_count, 200, 3
    d = inputs.PAPER_IDEAL_LENGTH
    sizes = inputs.log_uniform_sizes(count, 50, 5000, seed=4)
    graphs = [inputs.random_tree_plus_edges(int(n), int(n) // 2, seed=4_000_000 + i)
              for i, n in enumerate(sizes)]
    # one upload: the graphs and the positions concatenated into single tensors
    rp_all = torch.from_numpy(np.concatenate([g.row_ptr for g in graphs])).to(dev)
    ci_all = torch.from_numpy(np.concatenate([g.col_idx for g in graphs])).to(dev)
    n_arr = np.array([g.n for g in graphs], dtype=np.int64)
    nnz_arr = np.array([g.nnz for g in graphs], dtype=np.int64)
    dev_graphs, ro, co = [], 0, 0
    for g in graphs:
        dev_graphs.append((rp_all[ro:ro + g.n + 1], ci_all[co:co + g.nnz]))
        ro += g.n + 1
        co += g.nnz
    nv = int(sizes.sum())
    voff = np.concatenate([[0], np.cumsum(n_arr)[:-1]]).astype(np.int64)
    pos0 = torch.empty((nv, 2), dtype=torch.float32, device=dev)
    views = []
    for i, g in enumerate(graphs):
        v = pos0[voff[i]:voff[i] + g.n]
        gila.init_positions(g.n, i, inputs.PAPER_FRAME, inputs.PAPER_FRAME, gila.FP32, v)
        views.append(v)
    pos = torch.empty_like(pos0)
    pviews = [pos[voff[i]:voff[i] + g.n] for i, g in enumerate(graphs)]
    params = [gila.LayoutParams(temperature=gila.paper_schedule(g.n, 1.0, d, H), ideal_length=d,
                                precision=gila.FP32) for g in graphs]
    bparams = gila.BatchParams([p.temperature for p in params], d, gila.FP32)
    torch.cuda.synchronize()

    # the tuner's table (lanes per vertex by row-length class), taken once on
    # this batch and applied to every step's handle: each graph's plan is
    # then fixed and its bits reproducible
    b = gila.Batch.concatenated(rp_all, ci_all, n_arr, nnz_arr, k)
    default_lanes, cls = b.plan()
    table = b.tune(gila.FP32)
    tuned_lanes, _ = b.plan()      # the table by class, small graphs raised to fill
    b.free()

    def one_step():
        pos.copy_(pos0)
        b = gila.Batch.concatenated(rp_all, ci_all, n_arr, nnz_arr, k)
        b.set_plan(tuned_lanes)
        st = b.run(bparams, (pos, voff))
        return b, st

    for _ in range(warmup):
        b, _ = one_step()
        b.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b, st = one_step()
        info = b.info()
        lat = b.latency_ms()
        b.free()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    assert all(s.iterations_run == H for s in st)
    P = info["total_pairs"]
    nnz = sum(g.nnz for g in graphs)
    inter = (P + nnz) * H
    # run-only time (lists already built)
    b = gila.Batch.concatenated(rp_all, ci_all, n_arr, nnz_arr, k)
    b.set_plan(tuned_lanes)
    pos.copy_(pos0)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    b.run(bparams, (pos, voff))
    torch.cuda.synchronize()
    run_s = time.perf_counter() - tr0
    b.free()
    # plain per-graph solver on a sample, scaled by pair count
    sample = list(range(0, count, max(1, args.per_graph_every)))
    sp = 0
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for i in sample:
        pviews[i].copy_(views[i])
        gila.layout(dev_graphs[i][0], dev_graphs[i][1], k, params[i], pviews[i])
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - ts0
    for i in sample:
        kh = gila.build_khop(dev_graphs[i][0], dev_graphs[i][1], k)
        sp += (kh.info()["total_pairs"] + graphs[i].nnz) * H
        kh.free()
    per_graph_rate = sp / sample_s
    value = inter * steps / total_s
    p50, p99 = _percentiles(lat)
    # the persistent launch on the device clock: first graph's start to the
    # last graph's end
    launch_ms = float(np.max(lat))
    launch_bytes = algorithmic_bytes_per_iter(P, nnz, nv, 8) * H
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    return {
        "config": {"workload": f"batch{count}_tree+0.5n_k{k}_fp32_{H}iters",
                   "graphs": count, "n_range": [50, 5000], "vertices": nv, "edges": nnz // 2,
                   "k": k, "iterations": H, "total_pairs": P, "precision": "f32",
                   "data": "synthetic: random recursive tree + floor(n/2) extra edges per graph, "
                           "n log-uniform, init uniform in [0,1200)^2"},
        "interactions_per_s": value,
        "steps": steps, "warmup": warmup,
        "ms_per_step": total_s / steps * 1e3,
        "run_only_ms": run_s * 1e3,
        "latency_ms_within_launch": {"p50": p50, "p99": p99, "max": launch_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(TRAFFIC_FILE_BATCH),
                     "kernel": "batch_layout_kernel<FP32>", "kernel_ms": launch_ms,
                     "algorithmic_bytes_per_launch": launch_bytes},
        "per_graph_solver": {"interactions_per_s": per_graph_rate,
                             "sample_graphs": len(sample),
                             "speedup_of_batch": value / per_graph_rate},
        "plan": {"tuned_lanes_by_class": [int(x) for x in table],
                 "graphs_by_class": [int((cls == c).sum()) for c in range(8)],
                 "graphs_by_lanes": {str(int(l)): int((tuned_lanes == l).sum())
                                     for l in np.unique(tuned_lanes)}},
    }


def bench_batch(args) -> int:
    """The batched form on its own line (see batched_leg)."""
    r = batched_leg(args, args.steps, args.warmup)
    out = {
        "metric": "batched layout: k-hop force interactions/s over 4096 graphs",
        "value": r["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": r["config"], "run_only_ms": r["run_only_ms"],
        "latency_ms_within_batch": r["latency_ms_within_launch"], "roofline": r["roofline"],
        "per_graph_solver": r["per_graph_solver"], "plan": r["plan"],
    }
    print(json.dumps(with_traffic_rate(out)))
    return 0


def bench_serve(args) -> int:
    from paper_1606_02162_amd import serving_bench
    return serving_bench.main(args)


if __name__ == "__main__":
    sys.exit(main())
