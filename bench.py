"""Benchmark: Dynamic Frontier PageRank updates on one MI355X.

Workload (default): R-MAT graph with 2^22 vertices and 16 * 2^22 =
67,108,864 edges (a=0.57, b=c=0.19, seed 2), ranks from the GPU static
PageRank, then update batches of 1e-3 * |E| edges (80% insertions of
non-edges, 20% deletions of edges; seed 2020) applied one after another.
One step = apply one batch in place + one DF update (fp64, lock-free
persistent kernel by default).  Batches are resident in device memory
before the timed region.

Prints one JSON line with the metric, the roofline of the rank kernel
(algorithmic bytes counted by the library / kernel time from HIP events on
the library's stream) and the fp64 CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("update latency ms/batch + edges-processed/s & HBM GB/s; "
          "p50/p99 served latency")
PEAK_HBM_GBS = 8000.0
FRACS = [1e-7, 1e-5, 1e-3, 1e-1]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22",
                    choices=["rmat22", "rmat14", "grid4096"])
    ap.add_argument("--frac", type=float, default=1e-3)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--mode", default="async", choices=["async", "sync"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-static", action="store_true")
    ap.add_argument("--param", action="append", default=[],
                    help="library parameter override name=value")
    return ap.parse_args()


def load_workload(name):
    from paper_2407_19562_amd import inputs
    if name == "rmat22":
        n, s, d = inputs.cached("rmat_large", inputs.rmat_large)
        desc = "R-MAT 2^22 vertices, 67,108,864 edges (a=.57,b=c=.19), seed 2"
    elif name == "rmat14":
        n, s, d = inputs.cached("rmat_small", inputs.rmat_small)
        desc = "R-MAT 2^14 vertices, 131,072 edges (a=.57,b=c=.19), seed 1"
    else:
        n, s, d = inputs.cached("road_grid", inputs.road_grid)
        desc = "4096x4096 road-like grid, 5% pairs removed, 1e-4 long-range, seed 3"
    return n, s, d, desc


def batch_seed(name, frac):
    base = {"rmat22": 2000, "rmat14": 1000, "grid4096": 3000}[name]
    fi = FRACS.index(frac) if frac in FRACS else 9
    return base + 10 * fi


def traffic_record(kernel_tag):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2407_19562_amd", "csrc", "dfpr_rank.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
    if kv.get("kernel_source_sha1") != sha:
        return None
    try:
        return float(kv["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(n, s, d, seconds, desc):
    import oracle
    threads = os.cpu_count() or 1
    # calibrate with one sweep, then run a bounded sample
    m, t1, _ = oracle.timed_sweeps(n, s, d, 1, threads=threads)
    sweeps = max(1, int(seconds / max(t1, 1e-3)))
    m, t, tb = oracle.timed_sweeps(n, s, d, sweeps, threads=threads)
    return {"value": m * sweeps / t, "unit": "edges/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sweeps} fp64 Jacobi sweeps of Eq. 1 (static oracle) over "
                      f"{desc} plus self-loops ({m} edges/sweep), {t:.1f} s, "
                      f"CSR build ({tb:.1f} s) excluded"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the "
              "multi-GPU design is described in DESIGN.md and not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2407_19562_amd import dfpr, inputs
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)

    t0 = time.time()
    n, s, d, desc = load_workload(args.workload)
    log(f"workload {desc}: generated in {time.time() - t0:.1f}s")
    nb = args.warmup + args.steps
    batches = inputs.batches(n, s, d, nb, seed=batch_seed(args.workload, args.frac),
                             frac=args.frac)
    dev = [tuple(torch.from_numpy(a).cuda() for a in
                 (b.del_src, b.del_dst, b.ins_src, b.ins_dst)) for b in batches]
    overrides = {}
    for kv in args.param:
        k, v = kv.split("=")
        overrides[k] = float(v) if k in ("alpha", "tol", "frontier_tol") else int(v)
    mode = dfpr.DFPR_ASYNC if args.mode == "async" else dfpr.DFPR_SYNC
    stream = torch.cuda.current_stream()
    g = dfpr.Graph(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(),
                   precision=args.precision, mode=mode,
                   renormalize=int(args.precision == 32), **overrides)
    log(f"graph on device: {dfpr.dfpr_graph_bytes(g.h) / 2**30:.2f} GiB")
    rc, st = g.static()
    static_ms = st.ms
    static_sweeps = st.sweeps
    log(f"static: rc={rc} iters={st.sweeps} ms={st.ms:.2f}")

    def step(b):
        ad, ai = g.apply_batch(*b)
        rc, st = g.update()
        if rc < 0:
            raise RuntimeError(f"update failed {rc}")
        return ad, ai, st

    for i in range(args.warmup):
        step(dev[i])
    torch.cuda.synchronize()
    lat, upd, kern, edges, byts, sweeps, aff, launches = [], [], [], [], [], [], [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        ad, ai, st = step(dev[args.warmup + i])
        lat.append((time.perf_counter() - ts) * 1e3)
        b, nl = g.kernel_bytes()
        upd.append(st.ms)
        kern.append(st.ms_kernel)
        edges.append(st.edges_gathered)
        byts.append(b)
        launches.append(max(nl, 1))
        sweeps.append(st.sweeps)
        aff.append(st.affected)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    log(f"steps: latency ms {[round(x, 2) for x in lat]} sweeps {sweeps} affected {aff}")

    # stream-copy calibration of the achievable HBM bandwidth
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    bb = torch.empty_like(a)
    dfpr.dfpr_stream_copy(bb, a, nbytes)
    cms = min(dfpr.dfpr_stream_copy(bb, a, nbytes) for _ in range(3))
    copy_gbs = 2 * nbytes / (cms * 1e-3) / 1e9
    del a, bb

    # per launch of the rank kernel (one per update when async, one per
    # iteration when synchronous)
    kern_avg_ms = sum(kern) / sum(launches)
    bytes_avg = sum(byts) / sum(launches)
    achieved = bytes_avg / (kern_avg_ms * 1e-3) / 1e9
    tag = f"df_{args.mode}_{args.workload}_fp{args.precision}"
    hbm = traffic_record(tag)
    kname = "k_df_async" if args.mode == "async" else "k_sync_iter"
    result = {
        "metric": METRIC,
        "value": sum(edges) / total_s,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "batch": f"{args.frac:g}*|E| per step, 80% "
                   "insertions / 20% deletions, applied in sequence",
                   "update": f"dynamic frontier, {args.mode}, tol 1e-10, "
                   "frontier tol 1e-13, alpha 0.85"},
        "update_latency_ms": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99)),
                              "mean": statistics.mean(lat)},
        "update_device_ms_mean": statistics.mean(upd),
        "apply_ms_mean": statistics.mean(lat) - statistics.mean(upd),
        "edges_gathered_per_step": statistics.mean(edges),
        "sweeps_per_step": statistics.mean(sweeps),
        "affected_per_step": statistics.mean(aff),
        "static_recompute_ms": None if args.no_static else static_ms,
        "static_iters": static_sweeps,
        "copy_peak_gbs": copy_gbs,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": hbm,
                     "bytes_per_launch": bytes_avg,
                     "launch_ms": kern_avg_ms},
    }
    g.close()
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(n, s, d, args.cpu_seconds, desc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
