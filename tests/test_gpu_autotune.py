"""The autotuner: trial updates must leave every graph's edge set and ranks
as they were, the winner must come from the space, and updates after
tuning must still match the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2407_19562_amd import inputs

FP64_TOL = 1e-9


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


def keys(n, s, d):
    return np.sort(s.astype(np.int64) * n + d)


def test_tune_single_sync_graph(D, O):
    say("autotune sync")
    from paper_2407_19562_amd import autotune
    n, s, d = inputs.heavy_rows()
    R0, _, _ = O.pagerank(n, s, d)
    space = [{"split_min_degree": 64, "block_size": 128},
             {"split_min_degree": 4096, "block_size": 256}]
    with D.Graph(n, s, d, mode=D.DFPR_SYNC) as g:
        g.set_ranks(R0)
        best, table = autotune.tune(g, space=space, frac=1e-3, seed=5)
        assert best in space and len(table) == len(space)
        assert g.params.split_min_degree == best["split_min_degree"]
        assert np.array_equal(g.ranks(), R0)
        es, ed = g.edges(D.DFPR_OUT)
        assert np.array_equal(keys(n, es, ed), keys(n, s, d))
        b = inputs.batches(n, s, d, 1, 91, frac=1e-3)[0]
        ns, nd, res, ndel, nins = O.update(n, s, d, b, R0)
        ref, _, _ = O.pagerank(n, ns, nd)
        assert g.apply(b) == (ndel, nins)
        rc, st = g.update()
        assert rc == D.DFPR_OK
        assert float(np.abs(g.ranks() - ref).max()) < FP64_TOL


def test_tune_many_graphs(D, O):
    say("autotune batched")
    from paper_2407_19562_amd import autotune
    gs, refs = [], []
    try:
        for kind, n, s, d in inputs.graph_mix(6, 321, m_lo=500, m_hi=20000):
            R0, _, _ = O.pagerank(n, s, d)
            g = D.Graph(n, s, d)
            g.set_ranks(R0)
            gs.append(g)
            refs.append((n, s, d, R0))
        space = [{"chunk": 256, "block_size": 64}, {"chunk": 1024, "block_size": 256}]
        best, table = autotune.tune(gs, space=space, frac=1e-2, seed=7)
        assert best in space
        for g, (n, s, d, R0) in zip(gs, refs):
            assert np.array_equal(g.ranks(), R0)
            es, ed = g.edges(D.DFPR_OUT)
            assert np.array_equal(keys(n, es, ed), keys(n, s, d))
            assert g.params.chunk == best["chunk"]
    finally:
        for g in gs:
            g.close()
