"""Many graphs' updates in one persistent launch (dfpr_update_many):
every graph's ranks must match its own oracle, and the same update run
alone must agree with it (the lock-free schedule is nondeterministic, so
results are compared to tolerance, not bit-exact: within the bar once the
stopping error along the rank-mass direction is taken out, and within twice
the bar as a whole, since each is within the bar of the fixed point; see
agreement.py)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from agreement import agree
from paper_2407_19562_amd import inputs

FP64_TOL = 1e-9
FP32_REL = 1e-6


@pytest.fixture(scope="module")
def D():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2407_19562_amd import dfpr
    dfpr._lib()
    return dfpr


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle._lib()
    return oracle


def mix(count, seed):
    out = []
    for kind, n, s, d in inputs.graph_mix(count, seed, m_lo=200, m_hi=20000):
        b = inputs.batches(n, s, d, 1, seed=seed + n, frac=0.01)[0]
        out.append((kind, n, s, d, b))
    return out


@pytest.mark.parametrize("prec", [64, 32])
def test_update_many_matches_oracle_and_alone(D, O, prec):
    print("batched", prec, flush=True)
    graphs = mix(24, seed=900)
    refs, starts, handles, alone = [], [], [], []
    for kind, n, s, d, b in graphs:
        R0, _, _ = O.pagerank(n, s, d)
        ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
        ref, _, _ = O.pagerank(n, ns, nd)
        refs.append(ref)
        starts.append(R0)
        # the same update alone
        with D.Graph(n, s, d, precision=prec) as g:
            g.set_ranks(R0)
            g.apply(b)
            rc, st = g.update()
            assert rc >= 0
            alone.append(g.ranks())
        g = D.Graph(n, s, d, precision=prec)
        g.set_ranks(R0)
        g.apply(b)
        handles.append(g)
    try:
        rc, stats = D.dfpr_update_many([g.h for g in handles])
        assert rc == D.DFPR_OK
        for g, ref, a, st in zip(handles, refs, alone, stats):
            R = g.ranks()
            assert st.converged and st.sweeps > 0
            if prec == 64:
                assert np.abs(R - ref).max() < FP64_TOL
                ok, perp, whole = agree(R, a, ref, FP64_TOL)
            else:
                scale = np.abs(ref).max()
                assert np.abs(R - ref).max() / scale < FP32_REL
                ok, perp, whole = agree(R, a, ref, FP32_REL, relative=True)
            # batched and alone: the same result up to the stopping error
            # along the rank-mass direction (agreement.py)
            assert ok, (perp, whole)
        # marks were consumed: a second batched call is a no-op
        before = [g.ranks() for g in handles]
        rc, stats = D.dfpr_update_many([g.h for g in handles])
        assert rc == D.DFPR_OK and all(st.sweeps == 0 for st in stats)
        for g, r in zip(handles, before):
            assert np.array_equal(g.ranks(), r)
    finally:
        for g in handles:
            g.close()


def test_update_many_skips_graphs_without_marks(D, O):
    print("batched skip", flush=True)
    graphs = mix(4, seed=77)
    handles = []
    try:
        for i, (kind, n, s, d, b) in enumerate(graphs):
            g = D.Graph(n, s, d)
            g.static()
            if i % 2 == 0:
                g.apply(b)
            handles.append((g, n, s, d, b, i % 2 == 0))
        before = [h[0].ranks() for h in handles]
        rc, stats = D.dfpr_update_many([h[0].h for h in handles])
        assert rc == D.DFPR_OK
        for (g, n, s, d, b, applied), r0, st in zip(handles, before, stats):
            if applied:
                ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
                ref, _, _ = O.pagerank(n, ns, nd)
                assert np.abs(g.ranks() - ref).max() < FP64_TOL
            else:
                assert st.sweeps == 0 and np.array_equal(g.ranks(), r0)
    finally:
        for h in handles:
            h[0].close()


def test_update_many_rejects_mixed_precision(D, O):
    kind, n, s, d, b = mix(1, seed=5)[0]
    with D.Graph(n, s, d, precision=64) as a, D.Graph(n, s, d, precision=32) as c:
        with pytest.raises(D.DfprError):
            D.dfpr_update_many([a.h, c.h])
        with pytest.raises(D.DfprError):
            D.dfpr_update_many([a.h, a.h])
