"""The allocation-free batched launch (dfpr_update_many_noalloc) against
the regular one (dfpr_update_many), through the C ABI: the same graphs,
starting ranks and batches give results within the parity bar of the oracle
that agree with each other (agreement.py), on two calls in a row, the second
with fewer and smaller graphs (the shared device workspace keeps the first
call's contents)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from agreement import agree
from paper_2407_19562_amd import inputs

FP64_TOL = 1e-9
FP32_REL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def close(prec, R, ref):
    if prec == 64:
        return float(np.abs(R - ref).max()) < FP64_TOL
    return float(np.abs(R - ref).max() / np.abs(ref).max()) < FP32_REL


@pytest.mark.parametrize("prec", [64, 32])
def test_noalloc_matches_update_many(D, O, prec):
    say("no-alloc batched launch", prec)
    graphs = list(inputs.graph_mix(20, 700, m_lo=300, m_hi=30000))
    # call 1: all graphs, 1% batches; call 2: the first 7 graphs, 0.2% batches
    for call, (count, frac) in enumerate([(len(graphs), 1e-2), (7, 2e-3)]):
        sets = {"regular": [], "noalloc": []}
        refs = []
        for i, (kind, n, s, d) in enumerate(graphs[:count]):
            R0, _, _ = O.pagerank(n, s, d)
            b = inputs.batches(n, s, d, 1, seed=70 + 100 * call + i, frac=frac)[0]
            ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
            refs.append(O.pagerank(n, ns, nd)[0])
            for key in sets:
                g = D.Graph(n, s, d, precision=prec, renormalize=int(prec == 32))
                g.set_ranks(R0)
                g.apply(b)
                sets[key].append(g)
        try:
            rc1, st1 = D.dfpr_update_many([g.h for g in sets["regular"]])
            rc2, st2 = D.dfpr_update_many_noalloc([g.h for g in sets["noalloc"]])
            assert rc1 == D.DFPR_OK and rc2 == D.DFPR_OK
            for a, b, ref, x, y in zip(sets["regular"], sets["noalloc"], refs, st1, st2):
                assert x.converged and y.converged
                Ra, Rb = a.ranks(), b.ranks()
                assert close(prec, Ra, ref) and close(prec, Rb, ref)
                # two lock-free runs: the same up to the stopping error
                # along the rank-mass direction (agreement.py)
                ok, perp, whole = agree(Rb, Ra, ref, FP64_TOL if prec == 64 else FP32_REL,
                                        relative=prec == 32)
                assert ok, (perp, whole)
            say("  call", call, "graphs", count, "sweeps",
                [y.sweeps for y in st2][:8], "ok")
        finally:
            for key in sets:
                for g in sets[key]:
                    g.close()


def test_noalloc_rejects_too_many_graphs(D):
    n, s, d = inputs.erdos_renyi(50, 200, seed=3)
    with D.Graph(n, s, d) as g:
        hs = [g.h] * (D.DFPR_NOALLOC_MAX_GRAPHS + 1)
        with pytest.raises(D.DfprError):
            D.dfpr_update_many_noalloc(hs)
