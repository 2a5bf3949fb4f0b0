"""Benchmark: Dynamic Frontier PageRank updates on one MI355X.

Default workload (the headline line): R-MAT graph with 2^22 vertices and
16 * 2^22 = 67,108,864 edges (a=0.57, b=c=0.19, seed 2), ranks from the
GPU static PageRank, then update batches of 1e-3 * |E| edges (80%
insertions of non-edges, 20% deletions of edges; seed 2020) applied one
after another.  One step = apply one batch in place + one DF update (fp64).
Batches are resident in device memory before the timed region.

Other workloads (one JSON line each): `sweep` (batch sizes 1e-7..1e-1 |E|
on the same R-MAT, DF vs static recompute, fp64 and fp32), `grid4096`
(4096x4096 road-like grid, lock-free vs synchronous, fp64 and fp32),
`batched1024` (1024 small graphs in one launch vs one by one), `serving`
(resident graphs under a Poisson stream of batches), `rmat14` (small R-MAT),
`faults` (delayed or stopped workgroups, barrier-based vs lock-free),
`traversal` (Dynamic Traversal vs Dynamic Frontier vs naive-dynamic),
`vertices` (vertex insertion and removal with rescaled ranks).

Every line states the error of its results against the oracle: after the
timed region, untimed, the oracle's fp64 fixed point of the final graph is
computed on the host (the batches of a run are disjoint true changes, so the
final edge set is the base graph minus all deletions plus all insertions)
and compared with the GPU's final ranks vertex by vertex (L-infinity; for
fp32 also relative to the largest rank).  The oracle is test
infrastructure: bench.py calls it only in this error leg and in the
cpu_baseline leg, never in the timed path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
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
MODES = {"sync": 1, "async": 0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22",
                    choices=["rmat22", "rmat14", "sweep", "grid4096",
                             "batched1024", "serving", "faults", "traversal", "vertices",
                             "ftol"])
    ap.add_argument("--frac", type=float, default=1e-3)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--mode", default="sync", choices=["async", "sync"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the untimed comparison with the oracle (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched1024: keep the default launch parameters")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--graphs", type=int, default=None,
                    help="graph count for batched1024 / serving")
    ap.add_argument("--requests", type=int, default=None,
                    help="update batches in the serving stream")
    ap.add_argument("--scheme", default="each", choices=["batched", "each"],
                    help="serving: one batched lock-free launch per round, or "
                         "barrier-based updates graph by graph")
    ap.add_argument("--max-graphs", type=int, default=8,
                    help="serving: graphs per round (0: all with queued requests)")
    ap.add_argument("--param", action="append", default=[],
                    help="library parameter override name=value")
    return ap.parse_args()


def overrides(args):
    out = {}
    for kv in args.param:
        k, v = kv.split("=")
        out[k] = float(v) if k in ("alpha", "tol", "frontier_tol") else int(v)
    return out


def load_workload(name):
    from paper_2407_19562_amd import inputs
    if name in ("rmat22", "sweep"):
        n, s, d = inputs.cached("rmat_large", inputs.rmat_large)
        desc = "R-MAT 2^22 vertices, 67,108,864 edges (a=.57,b=c=.19), seed 2"
    elif name == "rmat14":
        n, s, d = inputs.cached("rmat_small", inputs.rmat_small)
        desc = "R-MAT 2^14 vertices, 131,072 edges (a=.57,b=c=.19), seed 1"
    else:
        n, s, d = inputs.cached("road_grid", inputs.road_grid)
        desc = ("4096x4096 bidirectional grid, 5%% of pairs removed, 1e-4|E| "
                "long-range edges, seed 3 (%d edges)" % s.size)
    return n, s, d, desc


def batch_seed(name, frac):
    base = {"rmat22": 2000, "sweep": 2000, "rmat14": 1000, "grid4096": 3000}[name]
    fi = FRACS.index(frac) if frac in FRACS else 9
    return base + 10 * fi


def kernel_sha():
    """Hash of the rank kernels' sources (dfpr_rank.hip, then dfpr_common.h)."""
    h = hashlib.sha1()
    for f in ("dfpr_rank.hip", "dfpr_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2407_19562_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def traffic_record(tag):
    """HBM bytes per dispatch of the rank kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha1") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(n, s, d, seconds, desc):
    import oracle
    threads = os.cpu_count() or 1
    m, t1, _ = oracle.timed_sweeps(n, s, d, 1, threads=threads)
    sweeps = max(1, int(seconds / max(t1, 1e-3)))
    m, t, tb = oracle.timed_sweeps(n, s, d, sweeps, threads=threads)
    return {"value": m * sweeps / t, "unit": "edges/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sweeps} fp64 Jacobi sweeps of Eq. 1 (static oracle) over "
                      f"{desc} plus self-loops ({m} edges/sweep), {t:.1f} s, "
                      f"CSR build ({tb:.1f} s) excluded"}


def cpu_baseline_1thread(n, s, d, seconds):
    """The same oracle sweeps on one host thread (a shorter sample)."""
    import oracle
    m, t1, _ = oracle.timed_sweeps(n, s, d, 1, threads=1)
    sweeps = max(1, int(seconds / max(t1, 1e-3)))
    m, t, _ = oracle.timed_sweeps(n, s, d, sweeps, threads=1)
    return {"value": m * sweeps / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} fp64 Jacobi sweeps on one thread, {t:.1f} s"}


# --- oracle leg: error of the final ranks (untimed) ------------------------------

def oracle_graph(n, s, d, batch_lists):
    """Edge list after applying, in order, each list of batches in
    `batch_lists`.  The batches of one list are disjoint true changes of the
    graph they were drawn from (inputs.batches), so a list applies as its
    union; successive lists apply in sequence with set semantics."""
    import oracle
    for bl in batch_lists:
        if not bl:
            continue
        cat = [np.concatenate([getattr(b, f) for b in bl]) for f in
               ("del_src", "del_dst", "ins_src", "ins_dst")]
        s, d, _, _ = oracle.apply_batch(n, s, d, *cat)
    return s, d


def oracle_ranks(n, s, d):
    import oracle
    R, it, _ = oracle.pagerank(n, s, d, threads=os.cpu_count() or 0)
    return R


def error_vs(R, ref, prec):
    """L-infinity error against the oracle, and for fp32 also relative to
    the largest oracle rank.  Bars: fp64 1e-9 absolute; fp32 1e-6 of the
    largest rank, or the fp64 bar where that is looser (graphs whose largest
    rank is below ~6e-4: there the method's own error at tol 1e-10, up to
    alpha/(1-alpha) * tol, is above 1e-6 of the largest rank in any
    precision)."""
    e = float(np.abs(np.asarray(R) - ref).max())
    rel = e / float(np.abs(ref).max())
    if prec == 64:
        return {"linf": e, "bar": 1e-9, "ok": e <= 1e-9}
    return {"linf": e, "rel_linf": rel, "bar": "rel 1e-6 or abs 1e-9",
            "ok": rel <= 1e-6 or e <= 1e-9}


def copy_peak_gbs(torch, dfpr):
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    dfpr.dfpr_stream_copy(b, a, nbytes)
    ms = min(dfpr.dfpr_stream_copy(b, a, nbytes) for _ in range(3))
    return 2 * nbytes / (ms * 1e-3) / 1e9


def run_steps(g, dev_batches, warmup, steps, torch):
    """Applies warmup + steps batches (device arrays) with one update each;
    returns per-step records of the timed steps and the wall time."""
    def step(b):
        g.apply_batch(*b)
        rc, st = g.update()
        if rc < 0:
            raise RuntimeError(f"update failed {rc}")
        if rc != 0 or not st.converged:
            log(f"warning: update ended at the sweep cap (rc {rc})")
        by, nl = g.kernel_bytes()
        return st, by, max(nl, 1)

    for i in range(warmup):
        step(dev_batches[i])
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        st, by, nl = step(dev_batches[warmup + i])
        rec.append({"lat_ms": (time.perf_counter() - ts) * 1e3, "st": st,
                    "bytes": by, "launches": nl})
    torch.cuda.synchronize()
    return rec, time.perf_counter() - t0


def summarize(rec):
    lat = [r["lat_ms"] for r in rec]
    return {
        "latency_ms": {"p50": float(np.percentile(lat, 50)),
                       "p99": float(np.percentile(lat, 99)),
                       "mean": statistics.mean(lat)},
        "update_device_ms_mean": statistics.mean(r["st"].ms for r in rec),
        "sweeps_mean": statistics.mean(r["st"].sweeps for r in rec),
        "affected_mean": statistics.mean(r["st"].affected for r in rec),
        "edges_gathered_mean": statistics.mean(r["st"].edges_gathered for r in rec),
        "converged_steps": sum(1 for r in rec if r["st"].converged),
    }


def device_batches(torch, batches):
    return [tuple(torch.from_numpy(a).cuda() for a in
                  (b.del_src, b.del_dst, b.ins_src, b.ins_dst)) for b in batches]


# --- workloads ------------------------------------------------------------------

def headline(args, torch, dfpr, inputs):
    t0 = time.time()
    n, s, d, desc = load_workload(args.workload)
    log(f"workload {desc}: loaded in {time.time() - t0:.1f}s")
    nb = args.warmup + args.steps
    batches = inputs.batches(n, s, d, nb, seed=batch_seed(args.workload, args.frac),
                             frac=args.frac)
    dev = device_batches(torch, batches)
    ov = overrides(args)
    ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    results = {}
    for mode in ([args.mode] + [m for m in MODES if m != args.mode]):
        g = dfpr.Graph(n, ds, dd, precision=args.precision, mode=MODES[mode],
                       renormalize=int(args.precision == 32), **ov)
        rc, st = g.static()
        static_ms, static_iters = st.ms, st.sweeps
        log(f"[{mode}] static: iters={st.sweeps} ms={st.ms:.2f}; "
            f"graph {dfpr.dfpr_graph_bytes(g.h) / 2**30:.2f} GiB")
        rec, total_s = run_steps(g, dev, args.warmup, args.steps, torch)
        final = g.ranks()
        g.close()
        log(f"[{mode}] latency ms {[round(r['lat_ms'], 2) for r in rec]} "
            f"sweeps {[r['st'].sweeps for r in rec]}")
        results[mode] = (rec, total_s, static_ms, static_iters, final)

    rec, total_s, static_ms, static_iters, _ = results[args.mode]
    kern_ms = sum(r["st"].ms_kernel for r in rec) / sum(r["launches"] for r in rec)
    bytes_launch = sum(r["bytes"] for r in rec) / sum(r["launches"] for r in rec)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    tag = f"df_{args.mode}_{args.workload}_fp{args.precision}"
    kname = "k_df_async" if args.mode == "async" else "k_sync_iter"
    summ = summarize(rec)
    other = [m for m in MODES if m != args.mode][0]
    orec = results[other][0]
    result = {
        "metric": METRIC,
        "value": sum(r["st"].edges_gathered for r in rec) / total_s,
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
        "config": {"workload": desc,
                   "batch": f"{args.frac:g}*|E| per step, 80% insertions / 20% "
                            "deletions, applied in sequence",
                   "update": f"dynamic frontier, {args.mode} "
                             f"({'Algorithm 1, barrier per iteration' if args.mode == 'sync' else 'Algorithm 2 scheme, one persistent launch'}), "
                             "tol 1e-10, frontier tol 1e-13, alpha 0.85"},
        "update_latency_ms": summ["latency_ms"],
        "converged_steps": summ["converged_steps"],
        "update_device_ms_mean": summ["update_device_ms_mean"],
        "apply_ms_mean": summ["latency_ms"]["mean"] - summ["update_device_ms_mean"],
        "edges_gathered_per_step": summ["edges_gathered_mean"],
        "sweeps_per_step": summ["sweeps_mean"],
        "affected_per_step": summ["affected_mean"],
        "static_recompute_ms": static_ms,
        "static_iters": static_iters,
        other: {"update_latency_ms_mean": summarize(orec)["latency_ms"]["mean"],
                "update_device_ms_mean": summarize(orec)["update_device_ms_mean"],
                "sweeps_per_step": summarize(orec)["sweeps_mean"],
                "edges_gathered_per_step": summarize(orec)["edges_gathered_mean"],
                "converged_steps": summarize(orec)["converged_steps"]},
        "copy_peak_gbs": copy_peak_gbs(torch, dfpr),
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic_record(tag),
                     "bytes_per_launch": bytes_launch,
                     "launch_ms": kern_ms},
    }
    if not args.no_oracle_error:
        # every step's batch applied in sequence: the oracle's fixed point of
        # the final graph against each scheme's final ranks
        t1 = time.time()
        ref = oracle_ranks(n, *oracle_graph(n, s, d, [batches]))
        errs = {m: error_vs(results[m][4], ref, args.precision) for m in results}
        result["error_vs_oracle"] = dict(errs, graph=f"after all {nb} batches",
                                         ranks_from="GPU static PageRank of the base graph")
        result["linf_vs_oracle"] = errs[args.mode]["linf"]
        if args.precision == 32:
            result["rel_vs_oracle"] = errs[args.mode]["rel_linf"]
        log(f"oracle error {errs} ({time.time() - t1:.1f}s)")
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(n, s, d, args.cpu_seconds, desc)
        result["cpu_baseline"]["single_thread"] = cpu_baseline_1thread(
            n, s, d, args.cpu_seconds / 3)
    return result


def sweep(args, torch, dfpr, inputs):
    n, s, d, desc = load_workload("sweep")
    ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    ov = overrides(args)
    out = {}
    refs = {}
    for prec in (64, 32):
        for f in FRACS:
            bs = inputs.batches(n, s, d, 5, seed=batch_seed("sweep", f), frac=f)
            dev = device_batches(torch, bs)
            g = dfpr.Graph(n, ds, dd, precision=prec, mode=MODES[args.mode],
                           renormalize=int(prec == 32), **ov)
            g.static()
            upd, stat, sw, aff, conv = [], [], [], [], []
            for b in dev:
                ts = time.perf_counter()
                g.apply_batch(*b)
                rc, st = g.update()
                upd.append((time.perf_counter() - ts) * 1e3)
                sw.append(st.sweeps)
                aff.append(st.affected)
                # static recompute of the same updated graph, for comparison
                R = torch.empty(n, dtype=torch.float64, device="cuda")
                g.ranks(R)
                rc2, st2 = g.static()
                stat.append(st2.ms)
                g.set_ranks(R)
                conv.append(bool(st.converged))
            final = g.ranks()
            g.close()
            out[f"fp{prec}_f{f:g}"] = {"batch_edges": bs[0].size,
                                       "affected_mean": statistics.mean(aff),
                                       "df_ms_mean": statistics.mean(upd),
                                       "static_ms_mean": statistics.mean(stat),
                                       "speedup_vs_static": statistics.mean(stat) / statistics.mean(upd),
                                       "sweeps_mean": statistics.mean(sw),
                                       "converged_steps": sum(conv)}
            if not args.no_oracle_error:
                if f not in refs:
                    refs[f] = oracle_ranks(n, *oracle_graph(n, s, d, [bs]))
                out[f"fp{prec}_f{f:g}"]["error_vs_oracle"] = error_vs(final, refs[f], prec)
            log(f"fp{prec} f={f:g}: {out[f'fp{prec}_f{f:g}']}")
    return {"metric": METRIC, "workload": "sweep", "config": {"workload": desc,
            "update": args.mode, "batches_per_size": 5,
            "error_vs_oracle": "final ranks after the 5 batches of a size"},
            "unit": "ms", "results": out}


def grid(args, torch, dfpr, inputs):
    n, s, d, desc = load_workload("grid4096")
    bs = inputs.batches(n, s, d, 5, seed=3000, frac=1e-4)
    dev = device_batches(torch, bs)
    ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    ov = overrides(args)
    out = {}
    roof = {}
    ref = None
    if not args.no_oracle_error:
        ref = oracle_ranks(n, *oracle_graph(n, s, d, [bs]))
    for prec in (64, 32):
        for mode in ("async", "sync"):
            g = dfpr.Graph(n, ds, dd, precision=prec, mode=MODES[mode],
                           renormalize=int(prec == 32), **ov)
            rc, st = g.static()
            rec, total_s = run_steps(g, dev, 0, len(dev), torch)
            final = g.ranks()
            g.close()
            sm = summarize(rec)
            key = f"{mode}_fp{prec}"
            out[key] = {"update_ms_mean": sm["latency_ms"]["mean"],
                        "update_device_ms_mean": sm["update_device_ms_mean"],
                        "sweeps_mean": sm["sweeps_mean"],
                        "affected_mean": sm["affected_mean"],
                        "edges_gathered_mean": sm["edges_gathered_mean"],
                        "converged_steps": sm["converged_steps"],
                        "static_ms": st.ms}
            if ref is not None:
                out[key]["error_vs_oracle"] = error_vs(final, ref, prec)
            # the rank kernel of each scheme against the HBM roofline
            kern_ms = sum(r["st"].ms_kernel for r in rec) / sum(r["launches"] for r in rec)
            by = sum(r["bytes"] for r in rec) / sum(r["launches"] for r in rec)
            kname = "k_df_async" if mode == "async" else "k_sync_iter"
            ach = by / (kern_ms * 1e-3) / 1e9
            roof[key] = {"bound": "hbm", "kernel": kname, "achieved": ach,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                         "traffic": traffic_record(f"df_{mode}_grid4096_fp{prec}"),
                         "bytes_per_launch": by, "launch_ms": kern_ms}
            log(f"{key}: {out[key]} roofline {roof[key]}")
    return {"metric": METRIC, "workload": "grid4096", "unit": "ms",
            "config": {"workload": desc, "batch": "1e-4*|E| (80/20), 5 in sequence"},
            "results": out, "roofline": roof["sync_fp64"], "roofline_all": roof,
            "copy_peak_gbs": copy_peak_gbs(torch, dfpr)}


def faults(args, torch, dfpr, inputs):
    """Fault simulation on the 2^22 R-MAT (DF, fp64, 1e-3 batches): a share
    of the rank kernels' workgroups sleeps after every claim, or stops at a
    claim boundary; barrier-based vs lock-free update time."""
    n, s, d, desc = load_workload("rmat22")
    bs = inputs.batches(n, s, d, 3, seed=batch_seed("rmat22", 1e-3), frac=1e-3)
    dev = device_batches(torch, bs)
    ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    ov = overrides(args)
    cases = {"none": [0], "delay_100us_1pct": [100] + [0] * 99,
             "delay_100us_10pct": [100] + [0] * 9, "stop_25pct": [-1, 0, 0, 0]}
    out = {}
    ref = None if args.no_oracle_error else oracle_ranks(n, *oracle_graph(n, s, d, [bs]))
    for mode in ("sync", "async"):
        for name, table in cases.items():
            g = dfpr.Graph(n, ds, dd, mode=MODES[mode], **ov)
            g.static()
            g.set_faults(table)
            rec, total_s = run_steps(g, dev, 0, len(dev), torch)
            final = g.ranks()
            g.close()
            sm = summarize(rec)
            out[f"{mode}_{name}"] = {"update_ms_mean": sm["latency_ms"]["mean"],
                                     "sweeps_mean": sm["sweeps_mean"],
                                     "converged_steps": sm["converged_steps"]}
            if ref is not None:
                out[f"{mode}_{name}"]["error_vs_oracle"] = error_vs(final, ref, 64)
            log(f"{mode} {name}: {out[f'{mode}_{name}']}")
    return {"metric": METRIC, "workload": "faults", "unit": "ms",
            "config": {"workload": desc, "batch": "1e-3*|E| (80/20), 3 in sequence",
                       "faults": "table entry per workgroup (w mod table length): "
                                 "sleep after every claim, or stop at a claim boundary"},
            "results": out}


def traversal(args, torch, dfpr, inputs):
    """Dynamic Traversal against Dynamic Frontier and naive-dynamic
    (barrier-based, fp64) on the 2^22 R-MAT and the road-like grid: per
    batch size, 3 batches in sequence from the same static ranks, one graph
    per method; time = apply + update wall time."""
    out = {}
    for name in ("rmat22", "grid4096"):
        n, s, d, desc = load_workload(name)
        ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
        ov = overrides(args)
        for f in (1e-7, 1e-5, 1e-3):
            bs = inputs.batches(n, s, d, 3, seed=batch_seed(name, f) + 5, frac=f)
            dev = device_batches(torch, bs)
            ref = None if args.no_oracle_error else oracle_ranks(n, *oracle_graph(n, s, d, [bs]))
            for method in ("df", "dt", "nd"):
                g = dfpr.Graph(n, ds, dd, mode=dfpr.DFPR_SYNC, **ov)
                g.static()
                lat, dev_ms, sweeps, aff, conv = [], [], [], [], []
                for b in dev:
                    torch.cuda.synchronize()
                    ts = time.perf_counter()
                    g.apply_batch(*b)
                    if method == "df":
                        rc, st = g.update()
                    elif method == "dt":
                        rc, st = g.update_traversal()
                    else:
                        rc, st = g.naive_dynamic()
                    lat.append((time.perf_counter() - ts) * 1e3)
                    if rc < 0:
                        raise RuntimeError(f"{method} failed {rc}")
                    dev_ms.append(st.ms)
                    sweeps.append(st.sweeps)
                    aff.append(n if method == "nd" else st.affected)
                    conv.append(bool(st.converged))
                final = g.ranks()
                g.close()
                key = f"{name}_f{f:g}_{method}"
                out[key] = {"ms_mean": statistics.mean(lat),
                            "device_ms_mean": statistics.mean(dev_ms),
                            "sweeps_mean": statistics.mean(sweeps),
                            "affected_mean": statistics.mean(aff),
                            "batch_edges": bs[0].size,
                            "converged_steps": sum(conv)}
                if ref is not None:
                    out[key]["error_vs_oracle"] = error_vs(final, ref, 64)
                log(f"{key}: {out[key]}")
    return {"metric": METRIC, "workload": "traversal", "unit": "ms",
            "config": {"workload": "R-MAT 2^22 (seed 2) and 4096x4096 road-like grid (seed 3)",
                       "batch": "f*|E| (80/20), 3 in sequence per size",
                       "methods": "df: Dynamic Frontier (Algorithm 1); dt: Dynamic "
                                  "Traversal (Algorithm 7); nd: naive-dynamic"},
            "results": out}


FTOLS = (1e-8, 1e-9, 1e-10, 1e-11, 1e-13, 1e-15)


def ftol_sweep(args, torch, dfpr, inputs):
    """The frontier tolerance tau_f (Section 4.4, tau / 1000 by default)
    against the work it causes and the error it leaves: the 2^22 R-MAT and
    the road-like grid, one batch of 1e-4|E| from the static ranks, each
    scheme, fp64; per tau_f the affected vertices, edges gathered, sweeps,
    update time and L-infinity error against the oracle's fixed point of
    the updated graph."""
    out = {}
    for name in ("rmat22", "grid4096"):
        n, s, d, desc = load_workload(name)
        ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
        ov = overrides(args)
        bs = inputs.batches(n, s, d, 1, seed=batch_seed(name, 1e-4) + 7, frac=1e-4)
        dev = device_batches(torch, bs)
        ref = None if args.no_oracle_error else oracle_ranks(n, *oracle_graph(n, s, d, [bs]))
        for mode in ("sync", "async"):
            g = dfpr.Graph(n, ds, dd, mode=MODES[mode], **ov)
            g.static()
            R0 = g.ranks()
            g.close()
            for ft in FTOLS:
                g = dfpr.Graph(n, ds, dd, mode=MODES[mode], frontier_tol=ft, **ov)
                g.set_ranks(R0)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                g.apply_batch(*dev[0])
                rc, st = g.update()
                ms = (time.perf_counter() - ts) * 1e3
                if rc < 0:
                    raise RuntimeError(f"update failed {rc}")
                final = g.ranks()
                g.close()
                key = f"{name}_{mode}_ftol{ft:g}"
                out[key] = {"ms": ms, "update_device_ms": st.ms, "sweeps": st.sweeps,
                            "affected": st.affected, "edges_gathered": st.edges_gathered,
                            "converged": bool(st.converged)}
                if ref is not None:
                    out[key]["error_vs_oracle"] = error_vs(final, ref, 64)
                log(f"{key}: {out[key]}")
    return {"metric": METRIC, "workload": "ftol", "unit": "ms",
            "config": {"workload": "R-MAT 2^22 (seed 2) and 4096x4096 road-like grid (seed 3)",
                       "batch": "1e-4*|E| (80/20), one batch from the static ranks",
                       "sweep": "frontier tolerance " + ", ".join(f"{x:g}" for x in FTOLS) +
                                " (tol 1e-10)"},
            "results": out}


def vertices(args, torch, dfpr, inputs):
    """Vertex insertion and removal on the 2^22 R-MAT (fp64, barrier-based
    DF): add k vertices with 16 in- and 16 out-edges each to random old
    vertices, or remove the k highest ids with their edges, then update;
    against a static recompute of the resulting graph.  k = 1e-5 n, 1e-4 n
    and 1e-3 n; times are wall times of each call."""
    n, s, d, desc = load_workload("rmat22")
    ds, dd = torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda()
    ov = overrides(args)
    out = {}
    rng = np.random.default_rng(4242)
    for frac in (1e-5, 1e-4, 1e-3):
        k = max(1, int(round(frac * n)))
        for op in ("add", "remove"):
            g = dfpr.Graph(n, ds, dd, mode=dfpr.DFPR_SYNC, reorder=0, **ov)
            g.static()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if op == "add":
                first = g.add_vertices(k)
                t1 = time.perf_counter()
                new = np.repeat(np.arange(first, first + k, dtype=np.int32), 16)
                old = rng.integers(0, n, new.size).astype(np.int32)
                b = inputs.Batch(np.empty(0, np.int32), np.empty(0, np.int32),
                                 np.concatenate([new, old]), np.concatenate([old, new]))
                g.apply(b)
            else:
                g.remove_vertices(k)
                t1 = time.perf_counter()
            t2 = time.perf_counter()
            rc, st = g.update()
            t3 = time.perf_counter()
            if rc < 0:
                raise RuntimeError(f"update failed {rc}")
            final = g.ranks()
            rc2, st2 = g.static()
            g.close()
            key = f"{op}_k{k}"
            out[key] = {"vertex_call_ms": (t1 - t0) * 1e3, "apply_ms": (t2 - t1) * 1e3,
                        "update_ms": (t3 - t2) * 1e3, "total_ms": (t3 - t0) * 1e3,
                        "sweeps": st.sweeps, "affected": st.affected,
                        "converged": bool(st.converged),
                        "static_ms": st2.ms, "static_iters": st2.sweeps}
            if not args.no_oracle_error:
                if op == "add":
                    n1 = n + k
                    fs, fd = oracle_graph(n1, s, d, [[b]])
                else:
                    n1 = n - k
                    keep = (s < n1) & (d < n1)
                    fs, fd = s[keep], d[keep]
                out[key]["error_vs_oracle"] = error_vs(final, oracle_ranks(n1, fs, fd), 64)
            log(f"{key}: {out[key]}")
    return {"metric": METRIC, "workload": "vertices", "unit": "ms",
            "config": {"workload": desc + ", caller order (reorder 0)",
                       "change": "add k vertices with 16 in- and 16 out-edges each, "
                                 "or remove the k highest ids with their edges"},
            "results": out}


def batched(args, torch, dfpr, inputs):
    count = args.graphs or 1024
    t0 = time.time()
    gl = list(inputs.graph_mix(count, 5000))
    log(f"{count} graphs generated in {time.time() - t0:.1f}s, "
        f"{sum(x[2].size for x in gl)} edges")
    ov = overrides(args)
    out = {}
    for prec in (64, 32):
        sets = []
        for _ in range(2):   # one set updated in one launch, one set one by one
            hs = []
            for g_i, (kind, n, s, d) in enumerate(gl):
                g = dfpr.Graph(n, s, d, precision=prec, mode=0,
                               renormalize=int(prec == 32), **ov)
                g.static()
                hs.append(g)
            sets.append(hs)
        if not args.no_autotune:
            # launch parameters from trial updates of the same graphs (their
            # edge sets and ranks are restored afterwards)
            from paper_2407_19562_amd import autotune
            t0 = time.perf_counter()
            try:
                best, table = autotune.tune(sets[0], frac=0.01, seed=777, refresh=True)
            except RuntimeError as exc:  # no candidate converged: keep defaults
                log(f"fp{prec} autotune failed: {exc}")
                out[f"fp{prec}_autotune"] = {"error": str(exc)}
                best, table = None, []
            # the one-by-one set keeps the library defaults, which suit
            # single small graphs
            default = {"split_min_degree": 0, "chunk": 0, "block_size": 0}
            t_def = [t for t, c in table if c == default]
            t_best = min((t for t, _ in table), default=math.inf)
            if best is not None:
                out[f"fp{prec}_autotune"] = {
                    "best": best, "seconds": time.perf_counter() - t0,
                    "default_trial_ms": t_def[0] * 1e3 if t_def else None,
                    "best_trial_ms": t_best * 1e3,
                    "gain_vs_default": (t_def[0] / t_best) if t_def else None,
                    "trials_ms": [(round(t * 1e3, 1) if t != math.inf else None, c)
                                  for t, c in table]}
                log(f"fp{prec} autotune: {best}")
        for g_i, (kind, n, s, d) in enumerate(gl):
            b = inputs.batches(n, s, d, 1, seed=5000 + g_i, frac=0.01)[0]
            for hs in sets:
                hs[g_i].apply(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, stats = dfpr.dfpr_update_many([g.h for g in sets[0]])
        t_batched = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        for g in sets[1]:
            rc1, g.last_stats = g.update()
        t_seq = (time.perf_counter() - t) * 1e3
        edges = sum(st.edges_gathered for st in stats)
        diffs = [float(np.abs(a.ranks() - b.ranks()).max()) for a, b in zip(*sets)]
        err = {}
        if not args.no_oracle_error:
            # every graph against its own oracle fixed point, both launches
            worst = {"batched": 0.0, "sequential": 0.0}
            ok = True
            missed = []   # graphs outside their bar: which launch, and how far
            for g_i, (kind, n, s, d) in enumerate(gl):
                b = inputs.batches(n, s, d, 1, seed=5000 + g_i, frac=0.01)[0]
                ref = oracle_ranks(n, *oracle_graph(n, s, d, [[b]]))
                for key, hs in zip(("batched", "sequential"), sets):
                    e = error_vs(hs[g_i].ranks(), ref, prec)
                    worst[key] = max(worst[key], e["linf"])
                    if prec == 32:
                        worst[key + "_rel"] = max(worst.get(key + "_rel", 0.0), e["rel_linf"])
                    ok = ok and e["ok"]
                    if not e["ok"]:
                        missed.append({"graph": g_i, "kind": kind, "n": n, "edges": int(s.size),
                                       "launch": key, "max_rank": float(ref.max()),
                                       **{k: v for k, v in e.items() if k != "bar"}})
            err = {"error_vs_oracle": {"max_over_graphs_" + k: v for k, v in worst.items()},
                   "error_bar": "abs 1e-9" if prec == 64 else "rel 1e-6 or abs 1e-9",
                   "all_ok": ok, "graphs_outside_bar": missed}
        out[f"fp{prec}"] = {"batched_ms": t_batched, "sequential_ms": t_seq,
                            "speedup": t_seq / t_batched,
                            "edges_gathered": edges,
                            "edges_gathered_sequential": sum(g.last_stats.edges_gathered
                                                             for g in sets[1]),
                            "edges_per_s_batched": edges / (t_batched * 1e-3),
                            "max_abs_diff_batched_vs_alone": max(diffs),
                            "graphs_differing": sum(x > 0 for x in diffs),
                            "converged": sum(1 for st in stats if st.converged),
                            **err}
        log(f"fp{prec}: {out[f'fp{prec}']}")
        for hs in sets:
            for g in hs:
                g.close()
    return {"metric": METRIC, "workload": "batched1024", "unit": "ms",
            "config": {"workload": f"{count} graphs, edges log-uniform 1e3..1e6, "
                       "half R-MAT half G(n,m), avg degree log-uniform 4..32, "
                       "seeds 5001+g", "batch": "1% of each graph (80/20)"},
            "results": out}


def serving(args, torch, dfpr, inputs):
    from paper_2407_19562_amd import serving as srv

    def check(server, graphs, streams, sample=6):
        """Spot check after the last stream: the smallest `sample` graphs
        against their oracle fixed points (each stream's batches of a graph
        are disjoint true changes, applied stream after stream)."""
        order = sorted(range(len(graphs)), key=lambda i: graphs[i][1].size)[:sample]
        worst, ok = 0.0, True
        for i in order:
            n, s, d = graphs[i]
            lists = [[r.batch for r in st if r.graph == i] for st in streams]
            ref = oracle_ranks(n, *oracle_graph(n, s, d, lists))
            e = error_vs(server.graphs[i].ranks(), ref, 32)
            worst = max(worst, e["rel_linf"])
            ok = ok and e["ok"]
        return {"graphs_checked": order, "max_rel_linf": worst,
                "bar": "rel 1e-6 or abs 1e-9", "all_ok": ok}

    return srv.bench(args, torch, dfpr, inputs, log,
                     check=None if args.no_oracle_error else check)


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
    fn = {"rmat22": headline, "rmat14": headline, "sweep": sweep,
          "grid4096": grid, "batched1024": batched, "serving": serving,
          "faults": faults, "traversal": traversal, "ftol": ftol_sweep,
          "vertices": vertices}[args.workload]
    result = fn(args, torch, dfpr, inputs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
