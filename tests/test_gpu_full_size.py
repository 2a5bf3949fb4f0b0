"""Parity at full size, in the launch configurations bench.py times: the
2^22-vertex R-MAT with 67,108,864 edges (barrier-based DF in fp64 and fp32,
lock-free DF in fp64; default parameters: degree-sorted order for the
barrier-based scheme, 12 wavefronts per CU, pieces from in-degree 2048,
1024-vertex tiles) and the 4096 x 4096 road-like grid (barrier-based and
lock-free).  Every vertex is compared with the oracle:
  * the GPU's static ranks with the oracle's fixed point of G^0;
  * after one batch (the benchmark's first), the DF ranks with the oracle's
    fixed point of G^1, L-infinity <= 1e-9 in fp64, normwise relative
    <= 1e-6 in fp32.  The DF update starts from the GPU's static ranks, as
    the benchmark does;
  * the applied counts and the exact set of initially marked vertices
    (numpy set operations on the edge lists);
  * Eq. 1 at sampled vertices, recomputed in fp64 from the GPU's ranks and
    the edge set read back from the device (a check of the stored graph as
    much as of the ranks).
The oracle's fixed points are computed once per graph and batch (a few
seconds of multithreaded Jacobi sweeps each)."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2407_19562_amd import inputs

ALPHA = 0.85
FP64_TOL = 1e-9
FP32_REL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def eq1_at(v, n, src, dst, R):
    """(1 - alpha)/n + alpha * sum over in(v) with the self-loop, for the
    distinct vertices v, from the edge list: |out(u)| = out-degree + 1."""
    od = np.bincount(src, minlength=n).astype(np.float64) + 1.0
    c = R / od
    vs = np.sort(v)
    sel = np.zeros(n, bool)
    sel[vs] = True
    mask = sel[dst]
    slot = np.searchsorted(vs, dst[mask])
    sums = np.bincount(slot, weights=c[src[mask]], minlength=vs.size)
    r = (1 - ALPHA) / n + ALPHA * (sums + c[vs])
    return vs, r


CASES = [  # graph, scheme, precision, batch fraction, batch seed (as bench.py)
    ("rmat22", "sync", 64, 1e-3, 2020),
    ("rmat22", "sync", 32, 1e-3, 2020),
    ("rmat22", "async", 64, 1e-3, 2020),
    ("rmat22", "async", 32, 1e-3, 2020),
    ("grid4096", "sync", 64, 1e-4, 3000),
    ("grid4096", "async", 64, 1e-4, 3000),
]

_CACHE = {}


def workload(name, frac, seed):
    """Graph, first batch, and the oracle's fixed points before and after
    it, computed once per (graph, batch)."""
    key = (name, frac, seed)
    if key in _CACHE:
        return _CACHE[key]
    import oracle
    t0 = time.time()
    if name == "rmat22":
        n, s, d = inputs.cached("rmat_large", inputs.rmat_large)
        assert n == 1 << 22 and s.size == 1 << 26
    else:
        n, s, d = inputs.cached("road_grid", inputs.road_grid)
        assert n == 4096 * 4096
    b = inputs.batches(n, s, d, 1, seed=seed, frac=frac)[0]
    say(f"  {name}: generated in {time.time() - t0:.1f}s; oracle on G^0 ...")
    R0, it0, _ = oracle.pagerank(n, s, d)
    say(f"  oracle G^0: {it0} sweeps, {time.time() - t0:.1f}s; applying the batch ...")
    ns, nd, d_true, i_true = oracle.apply_batch(n, s, d, b.del_src, b.del_dst,
                                                b.ins_src, b.ins_dst)
    R1, it1, _ = oracle.pagerank(n, ns, nd)
    say(f"  oracle G^1: {it1} sweeps, {time.time() - t0:.1f}s")
    _CACHE.clear()  # one graph's arrays at a time
    _CACHE[key] = (n, s, d, b, R0, ns, nd, R1, int(d_true.size), int(i_true.size))
    return _CACHE[key]


def bar(prec, R, ref):
    """fp64: L-infinity; fp32: L-infinity relative to the largest rank."""
    e = float(np.abs(R - ref).max())
    return e if prec == 64 else e / float(np.abs(ref).max())


@pytest.mark.parametrize("name,mode,prec,frac,seed", CASES)
def test_full_size(name, mode, prec, frac, seed):
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2407_19562_amd import dfpr
    say("full size:", name, mode, prec)
    n, s, d, b, R0ref, ns, nd, R1ref, ndel, nins = workload(name, frac, seed)
    tol = FP64_TOL if prec == 64 else FP32_REL
    rng = np.random.default_rng(77)
    m = dfpr.DFPR_SYNC if mode == "sync" else dfpr.DFPR_ASYNC
    # as bench.py creates it: the scheme and precision chosen, every other
    # parameter at its default
    with dfpr.Graph(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(),
                    mode=m, precision=prec, renormalize=int(prec == 32)) as g:
        rc, st = g.static()
        assert rc == dfpr.DFPR_OK and st.converged
        R0 = g.ranks()
        e0 = bar(prec, R0, R0ref)
        say("  static", st.sweeps, "iterations; vs oracle", e0)
        assert e0 < tol
        vs, r = eq1_at(rng.choice(n, 3000, replace=False), n, s, d, R0)
        scale = 1.0 if prec == 64 else float(R0.max())
        assert np.abs(r - R0[vs]).max() / scale < tol
        assert g.apply(b) == (ndel, nins) == (b.del_src.size, b.ins_src.size)
        # initial marks: every source itself (self-loop) and its previous
        # and current out-neighbours
        sources = np.unique(np.concatenate([b.del_src, b.ins_src]))
        is_src = np.zeros(n, bool)
        is_src[sources] = True
        want = np.zeros(n, bool)
        want[sources] = True
        want[d[is_src[s]]] = True
        want[b.ins_dst] = True
        aff, cnt = g.marks()
        assert cnt == int(want.sum())
        assert np.array_equal(aff, want)
        say("  marks", cnt)
        rc, st = g.update()
        assert rc == dfpr.DFPR_OK and st.converged, st.as_dict()
        R1 = g.ranks()
        e1 = bar(prec, R1, R1ref)
        say("  DF", st.sweeps, "sweeps,", st.affected, "affected; vs oracle", e1)
        assert e1 < tol
        es, ed = g.edges(dfpr.DFPR_OUT)
        assert es.size == ns.size
        changed = np.flatnonzero(R1 != R0)
        pick = np.unique(np.concatenate([
            rng.choice(changed, min(2000, changed.size), replace=False),
            rng.choice(n, 1000, replace=False), sources[:500]]))
        vs, r = eq1_at(pick, n, es, ed, R1)
        assert np.abs(r - R1[vs]).max() / scale < tol
