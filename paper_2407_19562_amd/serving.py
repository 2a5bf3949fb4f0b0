"""Serving many resident graphs: update batches arrive as a stream and are
applied with continuous batching.

Every graph keeps its slack CSR and ranks resident on the device.  Requests
(one update batch for one graph) queue per graph in arrival order.  Requests are
admitted as they arrive (as long as free device memory covers their
staging).  A graph's queued batches are applied in FIFO order (at most
`coalesce` at a time; batches applied before one update accumulate their
marks, which is the same as applying their union) and then the graph is
updated.  Two schemes:
  each     (default) every graph is served independently: whenever a graph
           with queued requests is idle and fewer than `max_graphs` graphs
           are in flight, a worker thread applies and updates it on the
           graph's own stream (barrier-based scheme), so the graphs' work
           overlaps on the device; its requests complete when that update
           does.  No graph waits for another graph's update.
  batched  rounds: the graphs with queued requests (at most `max_graphs`,
           longest-waiting first) are applied and then updated together in
           one persistent lock-free launch (dfpr_update_many); requests
           complete when their round does, and those arriving during a
           round join the next one.
A request's latency runs from its arrival to its completion.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import dfpr, inputs


@dataclass
class Request:
    graph: int
    batch: inputs.Batch
    arrival: float            # seconds from the start of the run
    done: float = math.nan    # completion time
    round: int = -1


@dataclass
class Report:
    latencies_ms: list = field(default_factory=list)
    rounds: int = 0
    updates: int = 0
    wall_s: float = 0.0
    edges_gathered: int = 0
    batch_edges: int = 0
    admission_waits: int = 0
    slot_waits: int = 0       # graphs with queued requests left waiting
                              # because max_graphs were in flight
    not_converged: int = 0    # updates that ended at the sweep cap
    apply_s: float = 0.0      # time spent applying batches (batched scheme)
    update_s: float = 0.0     # time spent in rank updates (each scheme:
                              # the whole run, applies and updates
                              # overlapped)

    def summary(self):
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"requests": len(self.latencies_ms),
                "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
                "throughput_batches_per_s": len(self.latencies_ms) / max(self.wall_s, 1e-9),
                "throughput_batch_edges_per_s": self.batch_edges / max(self.wall_s, 1e-9),
                "edges_gathered_per_s": self.edges_gathered / max(self.wall_s, 1e-9),
                "rounds": self.rounds, "updates": self.updates,
                "admission_waits": self.admission_waits,
                "slot_waits": self.slot_waits,
                "not_converged": self.not_converged,
                "apply_s": self.apply_s, "update_s": self.update_s,
                "wall_s": self.wall_s}


class Server:
    """Resident graphs plus the continuous-batching loop.

    scheme "each" (default): graphs are served independently, at most
    `max_graphs` at a time (0: no limit), each from a worker thread on its
    own stream.  scheme "batched": rounds of at most `max_graphs` graphs
    updated together in one persistent lock-free launch
    (dfpr_update_many).  In both, the graphs whose oldest request has waited
    longest go first."""

    def __init__(self, graphs, precision: int = 32, coalesce: int = 16,
                 reserve_bytes: int = 1 << 30, scheme: str = "each",
                 max_graphs: int = 8, **params):
        if scheme not in ("batched", "each"):
            raise ValueError("scheme must be 'batched' or 'each'")
        self.scheme = scheme
        mode = dfpr.DFPR_ASYNC if scheme == "batched" else dfpr.DFPR_SYNC
        self.graphs = []
        self.streams = []
        self.pool = None
        if scheme == "each":
            # every graph on its own stream, and a round's graphs applied and
            # updated from worker threads, so their work overlaps on the
            # device (the library's calls release the interpreter lock)
            import concurrent.futures
            import torch
            self.pool = concurrent.futures.ThreadPoolExecutor(max(1, max_graphs or len(graphs)))
        for n, s, d in graphs:
            stream = None
            if scheme == "each":
                st = torch.cuda.Stream()
                self.streams.append(st)
                stream = dfpr.ctypes.c_void_p(st.cuda_stream)
            kw = dict(params)
            if scheme == "each":
                # graphs are driven from several threads at once: no HIP
                # graph capture, which other threads' device calls can
                # invalidate (the library would fall back to launching
                # the iterations one by one anyway)
                kw.setdefault("graph_replay", 0)
            g = dfpr.Graph(n, s, d, precision=precision, mode=mode,
                           renormalize=int(precision == 32), stream=stream, **kw)
            g.static()
            self.graphs.append(g)
        self.coalesce = coalesce
        self.max_graphs = max_graphs
        self.reserve = reserve_bytes
        # adjacency growth accounting for admission (per graph): insertions
        # admitted since the last growth, the spare slots left for them, and
        # the device bytes a growth of both adjacency arrays takes
        m = [int(s.size) for _, s, _ in graphs]
        self.inserted = [0] * len(m)
        self.slack = [spare_slots(x) for x in m]
        self.growth = [growth_bytes(x) for x in m]

    def close(self):
        if self.pool is not None:
            self.pool.shutdown()
        for g in self.graphs:
            g.close()

    def _free_bytes(self):
        try:
            import torch
            return torch.cuda.mem_get_info()[0]
        except Exception:
            return 1 << 62

    def _need(self, r):
        """Device bytes request r may take: its staging (48 bytes per batch
        edge: the batch arrays and both directions' sort keys) plus, when
        its insertions may overflow the spare slots its graph has left, one
        growth of both adjacency arrays.  Returns (bytes, grows)."""
        need = 48 * r.batch.size
        grows = self.inserted[r.graph] + int(r.batch.ins_src.size) > self.slack[r.graph]
        if grows:
            need += self.growth[r.graph]
        return need, grows

    def _admit(self, rep, pending, queues, t0, open_loop, idle=False):
        """Moves arrived requests whose device memory (staging and possible
        adjacency growth) fits in free memory, above the reserve, to their
        graphs' queues.  idle: nothing is queued or in flight, so nothing
        will free memory; the first arrived request is admitted anyway."""
        now = time.perf_counter() - t0
        free = None
        while pending and (not open_loop or pending[0].arrival <= now):
            r = pending[0]
            need, grows = self._need(r)
            if free is None:
                free = self._free_bytes()
            if need + self.reserve > free and not idle:
                rep.admission_waits += 1
                break
            idle = False
            free -= need
            i = r.graph
            if grows:
                # the library grows an array to at least twice its slots
                self.inserted[i] = 0
                self.slack[i] *= 2
                self.growth[i] *= 2
            self.inserted[i] += int(r.batch.ins_src.size)
            queues[i].append(pending.popleft())

    def _run_each(self, requests, open_loop: bool) -> Report:
        import concurrent.futures as cf
        rep = Report()
        queues = [collections.deque() for _ in self.graphs]
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        limit = self.max_graphs or len(self.graphs)
        inflight = {}                      # future -> (graph, requests)
        t0 = time.perf_counter()
        done = 0

        def work(i, take):
            g = self.graphs[i]
            for r in take:
                g.apply(r.batch)
            rc, st = g.update()
            if rc < 0:
                raise RuntimeError(f"update of graph {i} failed ({rc})")
            return st, time.perf_counter() - t0

        while done < len(requests):
            self._admit(rep, pending, queues, t0, open_loop,
                        idle=not inflight and not any(queues))
            busy = {i for i, _ in inflight.values()}
            idle = [i for i, q in enumerate(queues) if q and i not in busy]
            idle.sort(key=lambda i: queues[i][0].arrival)
            free_slots = max(0, limit - len(inflight))
            rep.slot_waits += max(0, len(idle) - free_slots)
            for i in idle[:free_slots]:
                take = [queues[i].popleft()
                        for _ in range(min(self.coalesce, len(queues[i])))]
                rep.batch_edges += sum(r.batch.size for r in take)
                inflight[self.pool.submit(work, i, take)] = (i, take)
            if not inflight:
                if pending:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            timeout = None
            if pending and open_loop:
                timeout = max(0.0, pending[0].arrival - (time.perf_counter() - t0))
            fin, _ = cf.wait(list(inflight), timeout=timeout,
                             return_when=cf.FIRST_COMPLETED)
            for f in fin:
                i, take = inflight.pop(f)
                st, end = f.result()
                rep.rounds += 1           # one dispatch per graph update
                rep.updates += 1
                rep.edges_gathered += st.edges_gathered
                rep.not_converged += 0 if st.converged else 1
                for r in take:
                    r.done = end
                    rep.latencies_ms.append((end - r.arrival) * 1e3)
                done += len(take)
        rep.wall_s = time.perf_counter() - t0
        rep.update_s = rep.wall_s
        return rep

    def run(self, requests, open_loop: bool = True) -> Report:
        """Serves `requests` (sorted by arrival).  open_loop: requests are
        released at their arrival times; otherwise all are available at 0."""
        if self.scheme == "each":
            return self._run_each(requests, open_loop)
        rep = Report()
        queues = [collections.deque() for _ in self.graphs]
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        done = 0
        while done < len(requests):
            self._admit(rep, pending, queues, t0, open_loop, idle=not any(queues))
            active = [i for i, q in enumerate(queues) if q]
            if self.max_graphs and len(active) > self.max_graphs:
                rep.slot_waits += len(active) - self.max_graphs
                # the graphs whose oldest request waits longest go first
                active.sort(key=lambda i: queues[i][0].arrival)
                active = sorted(active[:self.max_graphs])
            if not active:
                if pending:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            served = []
            take = {}
            for i in active:
                take[i] = [queues[i].popleft()
                           for _ in range(min(self.coalesce, len(queues[i])))]
                served.extend(take[i])
                rep.batch_edges += sum(r.batch.size for r in take[i])
            ta = time.perf_counter()
            for i in active:
                for r in take[i]:
                    self.graphs[i].apply(r.batch)
            tu = time.perf_counter()
            rc, stats = dfpr.dfpr_update_many([self.graphs[i].h for i in active])
            if rc < 0:
                raise RuntimeError(f"batched update failed ({rc})")
            rep.not_converged += sum(0 if st.converged else 1 for st in stats)
            rep.apply_s += tu - ta
            rep.update_s += time.perf_counter() - tu
            end = time.perf_counter() - t0
            rep.rounds += 1
            rep.updates += len(active)
            rep.edges_gathered += sum(st.edges_gathered for st in stats)
            for r in served:
                r.done = end
                r.round = rep.rounds
                rep.latencies_ms.append((end - r.arrival) * 1e3)
            done += len(served)
        rep.wall_s = time.perf_counter() - t0
        return rep


def spare_slots(m: int) -> int:
    """Insertions a graph of m edges takes before its adjacency may grow: the
    spare tail is a quarter of the array (rows also keep a little slack of
    their own, ignored here)."""
    return max(1, m // 4)


def growth_bytes(m: int) -> int:
    """Device bytes one growth of both int32 adjacency arrays of a graph of
    m edges takes: the new array (twice the slots, about 1.25 m each) next to
    the old one until the copy is done."""
    return 2 * 4 * 3 * (m + m // 4 + 64)


def make_stream(graph_sizes, count: int, seed: int, rate: float | None,
                lo: float = 1, hi: float = 1e5, ins_share: float = 0.8,
                edges_of=None):
    """Poisson stream: `count` requests, target graph uniform, size
    log-uniform in [lo, hi] edges (capped at 1% of the graph), arrivals
    with mean rate `rate` per second (None: all at t = 0).  `edges_of(g)`
    returns (n, src, dst) of graph g for drawing its batches."""
    rng = np.random.default_rng(seed)
    gids = rng.integers(0, len(graph_sizes), count)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), count))
    arrivals = (np.cumsum(rng.exponential(1.0 / rate, count)) if rate
                else np.zeros(count))
    per_graph = collections.defaultdict(list)
    for k in range(count):
        cap = max(1, graph_sizes[gids[k]] // 100)
        per_graph[int(gids[k])].append((k, int(min(cap, max(1, round(sizes[k]))))))
    reqs = [None] * count
    for gidx, items in per_graph.items():
        n, s, d = edges_of(gidx)
        total = sum(sz for _, sz in items)
        # draw the graph's batches together so they stay true changes when
        # applied in sequence (distinct deletions, distinct non-edges)
        pool = inputs.batches(n, s, d, 1, seed=seed * 1000 + gidx, size=total,
                              ins_share=ins_share)[0]
        di = ii = 0
        for k, sz in items:
            nd = sz - int(round(ins_share * sz))
            ni = sz - nd
            b = inputs.Batch(pool.del_src[di:di + nd], pool.del_dst[di:di + nd],
                             pool.ins_src[ii:ii + ni], pool.ins_dst[ii:ii + ni])
            di += nd
            ii += ni
            reqs[k] = Request(int(gids[k]), b, float(arrivals[k]))
    return reqs


def bench(args, torch, dfpr_mod, inputs_mod, log, check=None):
    """Serving benchmark: resident R-MAT graphs, closed-loop saturated
    throughput X, then open-loop Poisson streams at 0.5 X and 0.8 X.
    check(server, graphs, streams), if given, runs after the last stream
    and before the graphs are freed (streams: the request lists in the order
    they were served)."""
    count = args.graphs or 64
    nreq = args.requests or 20000
    t0 = time.time()
    graphs = list(inputs.resident_mix(count, 4000))
    log(f"{count} resident graphs generated in {time.time() - t0:.1f}s, "
        f"{sum(s.size for _, s, _ in graphs)} edges")
    sizes = [s.size for _, s, _ in graphs]
    srv = Server(graphs, precision=32, scheme=args.scheme, max_graphs=args.max_graphs)
    try:
        res = {}
        streams = []
        closed = make_stream(sizes, nreq, 4, None, edges_of=lambda g: graphs[g])
        streams.append(closed)
        rep = srv.run(closed, open_loop=False)
        X = rep.summary()["throughput_batches_per_s"]
        res["closed_loop"] = rep.summary()
        log(f"closed loop: {res['closed_loop']}")
        for frac in (0.5, 0.8):
            reqs = make_stream(sizes, nreq, 40 + int(frac * 10), frac * X,
                               edges_of=lambda g: graphs[g])
            streams.append(reqs)
            rep = srv.run(reqs, open_loop=True)
            res[f"open_loop_{frac}X"] = rep.summary()
            log(f"open loop {frac}X: {res[f'open_loop_{frac}X']}")
        checked = check(srv, graphs, streams) if check is not None else None
    finally:
        srv.close()
    o = res["open_loop_0.8X"]
    return {"metric": "p50/p99 served latency (update latency ms/batch)",
            "workload": "serving",
            "value": o["throughput_batches_per_s"], "unit": "batches/s",
            "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
            "config": {"graphs": f"{count} R-MAT graphs, n log-uniform 2^16..2^21, "
                       "avg degree log-uniform 8..32, seeds 4001+g",
                       "stream": f"{nreq} batches, sizes log-uniform 1..1e5 edges "
                       "(at most 1% of the graph), 80/20, target uniform",
                       "ranks": "fp32 storage and sums, fp64 change tests and "
                       "renormalisation", "coalesce": srv.coalesce,
                       "scheme": srv.scheme, "max_graphs": srv.max_graphs},
            "results": res, **({"error_vs_oracle": checked} if checked else {})}
