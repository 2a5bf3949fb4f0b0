"""Autotuner for the launch parameters of the rank kernels.

Each candidate parameter set is timed on trial updates of the caller's own
graphs: a small random batch (deletions of existing edges, insertions of
non-edges, drawn from the graph's current edge set) is applied and the
graph updated, then the inverse batch is applied and the graph updated
again, so the edge set ends where it started.  Ranks are saved before the
first trial and restored after the last one.  Tuning therefore leaves every
graph's edge set and ranks as they were; only the order of entries inside
slack-CSR rows may change, which moves rounding in the last bits.

Spaces:
  sync    one graph, barrier-based scheme: the in-degree at which rows are
          summed in pieces (split_min_degree) and the workgroup size.
  async   one graph or many in one persistent launch (lock-free scheme):
          the vertex-to-wavefront mapping (split_min_degree: rows below it
          share a wavefront's 256-vertex step, rows at or above it get one
          wavefront per 4096-edge piece; 0 = the library's choice), groups
          per claim (chunk / 256;
          0 = the library's choice) and the workgroup size (0 = the
          library's choice).

A trial that ends at the sweep cap (or fails) disqualifies its parameter
set.  Winners are cached per graph-shape bucket (scheme, precision, graph
count, log2 of the vertex and edge counts) in a JSON file
($DFPR_TUNE_CACHE, default ~/.cache/dfpr_autotune.json); tune() returns a
cached winner without trials unless refresh=True.

Call it between updates (no applied batch may be pending).  The winner is
set on every graph and returned with the table of timings.  If a trial
fails, the error propagates with the parameters restored but the edge set
as the failing trial left it.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import dfpr, inputs

SPACES = {
    "sync": [{"split_min_degree": s, "block_size": b}
             for s in (0, 8192, 16384) for b in (0, 256)],
    "async": [{"split_min_degree": s, "chunk": c, "block_size": b}
              for s in (0, 512, 2048)
              for c in (0, 1024, 4096) for b in (0, 64, 128, 256)],
}


def cache_path() -> str:
    return os.environ.get("DFPR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "dfpr_autotune.json"))


def shape_bucket(graphs, scheme: str) -> str:
    """Graph-shape bucket of a tuning call: scheme, precision, graph count
    (log2, rounded) and the rounded log2 of the total vertices and edges."""
    n = sum(g.n for g in graphs)
    m = sum(g.size()[1] for g in graphs)
    c = len(graphs)
    prec = graphs[0].params.precision
    return (f"{scheme}/fp{prec}/g{round(math.log2(c))}/n{round(math.log2(max(n, 1)))}"
            f"/m{round(math.log2(max(m, 1)))}")


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(key: str, best: dict) -> None:
    cache = _load_cache()
    cache[key] = best
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def trial_batches(g, frac: float, seed: int):
    """A batch drawn from g's current edges and its inverse."""
    s, d = g.edges(dfpr.DFPR_OUT)
    b = inputs.batches(g.n, s, d, 1, seed, frac=frac)[0]
    inv = inputs.Batch(b.ins_src, b.ins_dst, b.del_src, b.del_dst)
    return b, inv


def tune(graphs, space=None, frac: float = 1e-3, seed: int = 0,
         repeats: int = 1, refresh: bool = False, use_cache: bool = True):
    """Times every parameter set in `space` on trial updates of `graphs`
    (one dfpr.Graph, or a list updated together by dfpr_update_many) and
    keeps the fastest converged one.  Returns (best, [(seconds, params),
    ...]); a cached winner comes back with an empty table."""
    single = isinstance(graphs, dfpr.Graph)
    graphs = [graphs] if single else list(graphs)
    if not graphs:
        raise ValueError("no graphs to tune")
    batched = len(graphs) > 1
    sync = not batched and graphs[0].params.mode == dfpr.DFPR_SYNC
    scheme = "sync" if sync else "async"
    key = None
    if space is None:
        space = SPACES[scheme]
        if use_cache:
            key = shape_bucket(graphs, scheme)
            cached = _load_cache().get(key)
            if cached and not refresh:
                for g in graphs:
                    g.set_params(**cached)
                return dict(cached), []
    keys = sorted({k for cfg in space for k in cfg})
    before = [{k: getattr(g.params, k) for k in keys} for g in graphs]
    saved = [g.ranks() for g in graphs]
    trials = [trial_batches(g, frac, seed + i) for i, g in enumerate(graphs)]
    table = []
    try:
        for cfg in space:
            for g in graphs:
                g.set_params(**cfg)
            spent = 0.0
            converged = True
            for _ in range(repeats):
                for leg in (0, 1):
                    for g, tb in zip(graphs, trials):
                        g.apply(tb[leg])
                    t0 = time.perf_counter()
                    if batched:
                        rc, stats = dfpr.dfpr_update_many([g.h for g in graphs])
                    else:
                        rc, st = graphs[0].update()
                        stats = [st]
                    spent += time.perf_counter() - t0
                    converged = converged and rc == dfpr.DFPR_OK and all(
                        st.converged for st in stats)
            # a set that hits the sweep cap is not a candidate
            table.append((spent if converged else math.inf, dict(cfg)))
    except BaseException:
        for g, p in zip(graphs, before):
            g.set_params(**p)
        raise
    finally:
        for g, r in zip(graphs, saved):
            g.set_ranks(r)
    if all(math.isinf(t) for t, _ in table):
        for g, p in zip(graphs, before):
            g.set_params(**p)
        raise RuntimeError("no parameter set converged within the sweep cap")
    best = min(table, key=lambda t: t[0])[1]
    for g in graphs:
        g.set_params(**best)
    if key is not None:
        _store_cache(key, best)
    return best, table
