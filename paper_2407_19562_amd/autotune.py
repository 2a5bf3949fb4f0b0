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
          groups per claim (chunk / 256; 0 = the library's choice) and the
          workgroup size.

Call it between updates (no applied batch may be pending).  The winner is
set on every graph and returned with the table of timings.  If a trial
fails, the error propagates with the parameters restored but the edge set
as the failing trial left it.
"""
from __future__ import annotations

import time

from . import dfpr, inputs

SPACES = {
    "sync": [{"split_min_degree": s, "block_size": b}
             for s in (1024, 2048, 4096) for b in (128, 256)],
    "async": [{"chunk": c, "block_size": b}
              for c in (0, 256, 1024, 4096) for b in (64, 128, 256)],
}


def trial_batches(g, frac: float, seed: int):
    """A batch drawn from g's current edges and its inverse."""
    s, d = g.edges(dfpr.DFPR_OUT)
    b = inputs.batches(g.n, s, d, 1, seed, frac=frac)[0]
    inv = inputs.Batch(b.ins_src, b.ins_dst, b.del_src, b.del_dst)
    return b, inv


def tune(graphs, space=None, frac: float = 1e-3, seed: int = 0,
         repeats: int = 1):
    """Times every parameter set in `space` on trial updates of `graphs`
    (one dfpr.Graph, or a list updated together by dfpr_update_many) and
    keeps the fastest.  Returns (best, [(seconds, params), ...])."""
    single = isinstance(graphs, dfpr.Graph)
    graphs = [graphs] if single else list(graphs)
    if not graphs:
        raise ValueError("no graphs to tune")
    batched = len(graphs) > 1
    if space is None:
        sync = not batched and graphs[0].params.mode == dfpr.DFPR_SYNC
        space = SPACES["sync" if sync else "async"]
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
            for _ in range(repeats):
                for leg in (0, 1):
                    for g, tb in zip(graphs, trials):
                        g.apply(tb[leg])
                    t0 = time.perf_counter()
                    if batched:
                        dfpr.dfpr_update_many([g.h for g in graphs])
                    else:
                        graphs[0].update()
                    spent += time.perf_counter() - t0
            table.append((spent, dict(cfg)))
    except BaseException:
        for g, p in zip(graphs, before):
            g.set_params(**p)
        raise
    finally:
        for g, r in zip(graphs, saved):
            g.set_ranks(r)
    best = min(table, key=lambda t: t[0])[1]
    for g in graphs:
        g.set_params(**best)
    return best, table
