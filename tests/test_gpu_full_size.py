"""Parity at full size, in the launch configurations bench.py times: the
2^22-vertex R-MAT with 67,108,864 edges (barrier-based DF, fp64 and fp32,
default parameters: degree-sorted order, 12 wavefronts per CU, pieces from
in-degree 2048) and the 4096 x 4096 road-like grid (barrier-based and
lock-free).  The oracle's full iteration takes minutes on the host, so
the checks are the ones that hold at any size and are cheap to compute:
  * applied counts and the set of initially marked vertices are integers,
    compared exactly with numpy set operations on the edge lists;
  * Eq. 1 holds at sampled vertices: r_v recomputed in fp64 from the GPU's
    own ranks and the current edge set (read back) stays within the
    tolerance's reach of the stored rank, for the static ranks and again
    after a DF update (sampled among affected and unaffected vertices)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2407_19562_amd import inputs

ALPHA = 0.85


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
    ("grid4096", "sync", 64, 1e-4, 3000),
    ("grid4096", "async", 64, 1e-4, 3000),
]


@pytest.mark.parametrize("name,mode,prec,frac,seed", CASES)
def test_full_size(name, mode, prec, frac, seed):
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2407_19562_amd import dfpr
    say("full size:", name, mode, prec)
    if name == "rmat22":
        n, s, d = inputs.cached("rmat_large", inputs.rmat_large)
        assert n == 1 << 22 and s.size == 1 << 26
    else:
        n, s, d = inputs.cached("road_grid", inputs.road_grid)
        assert n == 4096 * 4096
    # fp64: Eq. 1 within the iteration tolerance's reach; fp32: normwise
    # relative 1e-6 (residual / largest rank)
    tol = 1e-9 if prec == 64 else 1e-6
    rng = np.random.default_rng(77)
    m = dfpr.DFPR_SYNC if mode == "sync" else dfpr.DFPR_ASYNC
    # as bench.py creates it: the scheme and precision chosen, every other
    # parameter at its default
    with dfpr.Graph(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(),
                    mode=m, precision=prec, renormalize=int(prec == 32)) as g:
        rc, st = g.static()
        assert rc == dfpr.DFPR_OK and st.converged
        R0 = g.ranks()
        scale = 1.0 if prec == 64 else float(R0.max())
        say("  static", st.sweeps, "iterations")
        vs, r = eq1_at(rng.choice(n, 3000, replace=False), n, s, d, R0)
        err0 = np.abs(r - R0[vs]).max() / scale
        say("  static Eq. 1 residual at samples", err0)
        assert err0 < tol
        b = inputs.batches(n, s, d, 1, seed=seed, frac=frac)[0]
        assert g.apply(b) == (b.del_src.size, b.ins_src.size)
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
        assert rc == dfpr.DFPR_OK and st.converged
        R1 = g.ranks()
        es, ed = g.edges(dfpr.DFPR_OUT)
        assert es.size == s.size - b.del_src.size + b.ins_src.size
        changed = np.flatnonzero(R1 != R0)
        pick = np.unique(np.concatenate([
            rng.choice(changed, min(2000, changed.size), replace=False),
            rng.choice(n, 1000, replace=False), sources[:500]]))
        vs, r = eq1_at(pick, n, es, ed, R1)
        err1 = np.abs(r - R1[vs]).max() / scale
        say("  DF", st.sweeps, "iterations,", changed.size, "ranks changed,",
            "Eq. 1 residual at samples", err1)
        assert err1 < tol
