"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerances: fp64 ranks within 1e-9 L-infinity of the oracle's fixed point
(the paper's DF error bound at tau = 1e-10, Sections 4.4 and 5.2.2); fp32
ranks within 1e-6 normwise relative (max |R32 - R*| / max |R*|).  Graph
structure (edge sets, applied counts, marks) is compared exactly.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2407_19562_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
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


def edge_keys(n, s, d):
    return np.sort(s.astype(np.int64) * n + d.astype(np.int64))


def err64(a, b):
    return float(np.abs(a - b).max())


def rel32(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def graph(D, n, s, d, **kw):
    return D.Graph(n, s, d, **kw)


# --- structure ------------------------------------------------------------------

@pytest.mark.parametrize("reorder", [0, 1])
@pytest.mark.parametrize("case", ["rmat_small", "ragged", "tiny", "empty"])
def test_structure_roundtrip(D, O, case, reorder):
    say("structure", case, reorder)
    if case == "rmat_small":
        n, s, d = inputs.rmat_small()
    elif case == "ragged":
        n, s, d = inputs.erdos_renyi(1000, 7000, seed=2)
        # duplicates and self pairs in the input are dropped
        s = np.concatenate([s, s[:50], np.arange(10, dtype=np.int32)])
        d = np.concatenate([d, d[:50], np.arange(10, dtype=np.int32)])
    elif case == "tiny":
        n, s, d = 3, np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    else:
        n, s, d = 5, np.empty(0, np.int32), np.empty(0, np.int32)
    ref = O.edge_set(n, s, d)
    with graph(D, n, s, d, reorder=reorder) as g:
        assert g.size() == (n, ref.size)
        for direction in (D.DFPR_OUT, D.DFPR_IN):
            gs, gd = g.edges(direction)
            assert np.array_equal(edge_keys(n, gs, gd), ref)


def test_apply_set_semantics(D, O):
    say("apply set semantics")
    n = 5
    s = np.array([0, 0, 1, 2], np.int32)
    d = np.array([1, 2, 2, 3], np.int32)
    ds, dd = np.array([0, 3, 2, 0], np.int32), np.array([1, 4, 2, 2], np.int32)
    is_, id_ = np.array([4, 4, 1, 3, 0], np.int32), np.array([0, 0, 2, 3, 2], np.int32)
    ns, nd, dt, it = O.apply_batch(n, s, d, ds, dd, is_, id_)
    with graph(D, n, s, d) as g:
        ad, ai = g.apply_batch(ds, dd, is_, id_)
        assert (ad, ai) == (dt.size, it.size)
        for direction in (D.DFPR_OUT, D.DFPR_IN):
            assert np.array_equal(edge_keys(n, *g.edges(direction)),
                                  edge_keys(n, ns, nd))


@pytest.mark.parametrize("kind,frac", [("rmat_small", 1e-3), ("rmat_small", 5e-2),
                                       ("rmat_small", 0.3), ("heavy_rows", 5e-2)])
def test_apply_batches_match_oracle(D, O, kind, frac):
    say("apply batches", kind, frac)
    n, s, d = getattr(inputs, kind)()
    bs = inputs.batches(n, s, d, 3, seed=31, frac=frac)
    cs, cd = s, d
    with graph(D, n, s, d) as g:
        for b in bs:
            cs, cd, dt, it = O.apply_batch(n, cs, cd, b.del_src, b.del_dst,
                                           b.ins_src, b.ins_dst)
            ad, ai = g.apply(b)
            assert (ad, ai) == (dt.size, it.size)
        for direction in (D.DFPR_OUT, D.DFPR_IN):
            assert np.array_equal(edge_keys(n, *g.edges(direction)),
                                  edge_keys(n, cs, cd))


def test_apply_row_relocation_and_growth(D, O):
    say("relocation")
    # a hub gains thousands of out- and in-edges: rows outgrow their slack
    # and the spare tail of the adjacency arrays has to grow
    n = 70000
    s = np.arange(1, 200, dtype=np.int32)
    d = np.zeros(199, np.int32)
    ins_s = np.concatenate([np.zeros(69000, np.int32), np.arange(1000, 69999, dtype=np.int32)])
    ins_d = np.concatenate([np.arange(1, 69001, dtype=np.int32), np.full(68999, 5, np.int32)])
    ns, nd, dt, it = O.apply_batch(n, s, d, [], [], ins_s, ins_d)
    with graph(D, n, s, d) as g:
        ad, ai = g.apply_batch(np.empty(0, np.int32), np.empty(0, np.int32), ins_s, ins_d)
        assert (ad, ai) == (0, it.size)
        for direction in (D.DFPR_OUT, D.DFPR_IN):
            assert np.array_equal(edge_keys(n, *g.edges(direction)),
                                  edge_keys(n, ns, nd))


def test_apply_long_rows(D, O):
    # rows of 4096+ entries are edited by whole workgroups: 3000 deletions
    # in one out-row (more keys than fit in LDS), 900 in one in-row, plus
    # insertions on the same rows; edge sets, counts and marks must match
    say("apply long rows")
    n, s, d = inputs.heavy_rows()
    rng = np.random.default_rng(12)
    hub_out, hub_in = 8, 5                 # out-degree 20000, in-degree 25000
    eo = np.flatnonzero(s == hub_out)
    ei = np.flatnonzero(d == hub_in)
    dsel = np.concatenate([rng.choice(eo, 3000, replace=False),
                           rng.choice(ei, 900, replace=False)])
    dsel = np.unique(dsel)
    keyset = set((s.astype(np.int64) * n + d).tolist())
    ins = []
    while len(ins) < 400:
        a, b = (hub_out, int(rng.integers(0, n))) if len(ins) % 2 else (int(rng.integers(0, n)), hub_in)
        if a != b and a * n + b not in keyset:
            keyset.add(a * n + b)
            ins.append((a, b))
    is_, id_ = (np.array(x, np.int32) for x in zip(*ins))
    ns, nd, dt, it = O.apply_batch(n, s, d, s[dsel], d[dsel], is_, id_)
    R, _, _ = O.pagerank(n, s, d)
    src = np.concatenate([dt // n, it // n]).astype(np.int32)
    ref = O.df_bb(n, (s, d), (ns, nd), src, R, max_iters=0)
    with graph(D, n, s, d) as g:
        ad, ai = g.apply_batch(s[dsel], d[dsel], is_, id_)
        assert (ad, ai) == (dt.size, it.size)
        for direction in (D.DFPR_OUT, D.DFPR_IN):
            assert np.array_equal(edge_keys(n, *g.edges(direction)),
                                  edge_keys(n, ns, nd))
        aff, cnt = g.marks()
        assert np.array_equal(aff, ref.affected)
        assert cnt == ref.initial_marked


def test_invalid_batch_is_rejected_whole(D, O):
    say("invalid batch")
    n, s, d = inputs.rmat(8, 1000, seed=3)
    with graph(D, n, s, d) as g:
        before = edge_keys(n, *g.edges())
        with pytest.raises(D.DfprError) as ei:
            g.apply_batch(np.array([0], np.int32), np.array([1], np.int32),
                          np.array([2, n], np.int32), np.array([3, 4], np.int32))
        assert ei.value.status == D.DFPR_EINVAL
        assert np.array_equal(edge_keys(n, *g.edges()), before)


# --- marking (Section 4.1.2, with self-loops) --------------------------------------

def test_marking_frontier_example(D, O):
    say("marking example")
    with open(os.path.join(GOLD, "frontier_example.json")) as f:
        ex = json.load(f)
    n = ex["n"]
    s, d = (np.array(x, np.int32) for x in zip(*ex["edges_before"]))
    with graph(D, n, s, d) as g:
        g.apply_batch(np.array([10], np.int32), np.array([11], np.int32),
                      np.array([7], np.int32), np.array([9], np.int32))
        aff, cnt = g.marks()
        # the narrative's {8, 9, 11} plus the sources 7 and 10 (self-loops)
        assert sorted(np.flatnonzero(aff).tolist()) == [7, 8, 9, 10, 11]
        assert cnt == 5


@pytest.mark.parametrize("kind,reorder", [("rmat_small", 0), ("rmat_small", 1),
                                          ("heavy_rows", 0)])
def test_marking_matches_oracle_rmat(D, O, kind, reorder):
    say("marking", kind, reorder)
    n, s, d = getattr(inputs, kind)()
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-2 if kind == "heavy_rows" else 1e-3)[0]
    R, _, _ = O.pagerank(n, s, d)
    ns, nd, dt, it = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
    src = np.concatenate([dt // n, it // n]).astype(np.int32)
    ref = O.df_bb(n, (s, d), (ns, nd), src, R, max_iters=0)
    with graph(D, n, s, d, reorder=reorder) as g:
        g.apply(b)
        aff, cnt = g.marks()
        assert np.array_equal(aff, ref.affected)
        assert cnt == ref.initial_marked


# --- ranks --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [64, 32])
def test_static_matches_oracle(D, O, prec):
    say("static", prec)
    n, s, d = inputs.rmat_small()
    ref, _, _ = O.pagerank(n, s, d)
    with graph(D, n, s, d, precision=prec, renormalize=int(prec == 32)) as g:
        rc, st = g.static()
        assert rc == D.DFPR_OK and st.converged
        R = g.ranks()
    if prec == 64:
        assert err64(R, ref) < FP64_TOL
        assert abs(R.sum() - 1) < 1e-8
    else:
        assert rel32(R, ref) < FP32_REL


_BASE_RANKS = {}


def base_graph(O, kind):
    """(n, src, dst, oracle ranks) of a named input, computed once."""
    if kind not in _BASE_RANKS:
        n, s, d = getattr(inputs, kind)()
        R0, _, _ = O.pagerank(n, s, d)
        _BASE_RANKS[kind] = (n, s, d, R0)
    return _BASE_RANKS[kind]


# rmat_mid (2^20 vertices) takes the large-graph paths: 1024-vertex tiles,
# and with reorder 2 the degree-sorted order (in the lock-free scheme also
# the interleaved group worklist, pieces from 512 in-edges and 4-group claims)
@pytest.mark.parametrize("kind,reorder", [("rmat_small", 0), ("rmat_small", 1),
                                          ("heavy_rows", 0), ("rmat_mid", 2)])
@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("frac", [1e-3, 1e-2])
def test_df_fp64_matches_oracle(D, O, mode, frac, kind, reorder):
    say("df fp64", kind, mode, frac, reorder)
    n, s, d, R0 = base_graph(O, kind)
    b = inputs.batches(n, s, d, 1, 1001, frac=frac)[0]
    ns, nd, res, ndel, nins = O.update(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    # the paper's cap of 500 sweeps in both schemes
    with graph(D, n, s, d, mode=m, reorder=reorder) as g:
        g.set_ranks(R0)                        # parity mode: R^{t-1} exact
        assert g.apply(b) == (ndel, nins)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        R = g.ranks()
    say("  err", err64(R, ref), "sweeps", st.sweeps, "affected", st.affected,
        "oracle iters", res.iters, "affected", int(res.affected.sum()))
    assert err64(R, ref) < FP64_TOL
    assert st.initial_marked == res.initial_marked
    if mode == "sync":
        # same algorithm as the oracle's Algorithm 1: same iteration count and
        # affected set up to the rounding of borderline frontier decisions
        assert abs(st.sweeps - res.iters) <= 1
        assert abs(st.affected - int(res.affected.sum())) <= max(3, res.affected.sum() // 1000)


def test_frontier_tolerance_sweep(D, O):
    # the frontier tolerance tau_f (Section 4.4) against the oracle's
    # Algorithm 1 at the same tau_f: the barrier-based update affects the
    # same vertices and ends at the same ranks for every tau_f; the error
    # against the fixed point grows once tau_f nears tau, and at the paper's
    # tau / 1000 both schemes meet the bar
    say("frontier tolerance sweep")
    n, s, d, R0 = base_graph(O, "rmat_small")
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-4)[0]
    ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
    ref, _, _ = O.pagerank(n, ns, nd)
    errs = {}
    for ft in (1e-8, 1e-9, 1e-10, 1e-13, 0.0):
        _, _, res, _, _ = O.update(n, s, d, b, R0, ftol=ft)
        with graph(D, n, s, d, mode=D.DFPR_SYNC, frontier_tol=ft) as g:
            g.set_ranks(R0)
            g.apply(b)
            rc, st = g.update()
            assert rc == D.DFPR_OK and st.converged
            R = g.ranks()
        say("  tau_f", ft, "affected", st.affected, int(res.affected.sum()),
            "err", err64(R, ref), err64(res.R, ref))
        assert abs(st.affected - int(res.affected.sum())) <= max(3, res.affected.sum() // 1000)
        assert err64(R, res.R) < FP64_TOL
        errs[ft] = err64(R, ref)
    assert errs[1e-8] > FP64_TOL >= errs[1e-13]
    with graph(D, n, s, d, mode=D.DFPR_ASYNC) as g:
        g.set_ranks(R0)
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and err64(g.ranks(), ref) < FP64_TOL


@pytest.mark.parametrize("kind", ["rmat_small", "heavy_rows"])
@pytest.mark.parametrize("prec", [64, 32])
def test_lock_free_stop_rules(D, O, kind, prec):
    # both stopping rules of the lock-free update meet the bar; the strict
    # reading of Algorithm 2 (every change above tau_f re-opens) never takes
    # fewer sweeps than the tolerance rule
    say("lock-free stop rules", kind, prec)
    n, s, d, R0 = base_graph(O, kind)
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-2)[0]
    ns, nd, res, ndel, nins = O.update(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    sweeps = {}
    for rule in (D.DFPR_STOP_TOL, D.DFPR_STOP_FRONTIER):
        with graph(D, n, s, d, mode=D.DFPR_ASYNC, precision=prec,
                   renormalize=int(prec == 32), lf_stop=rule) as g:
            g.set_ranks(R0)
            assert g.apply(b) == (ndel, nins)
            rc, st = g.update()
            assert rc == D.DFPR_OK and st.converged, st.as_dict()
            R = g.ranks()
        sweeps[rule] = st.sweeps
        say("  rule", rule, "sweeps", st.sweeps, "err", err64(R, ref))
        if prec == 64:
            assert err64(R, ref) < FP64_TOL
        else:
            assert rel32(R, ref) < FP32_REL
    assert sweeps[D.DFPR_STOP_FRONTIER] >= sweeps[D.DFPR_STOP_TOL]


@pytest.mark.parametrize("split", [1, 64, 2048, 1 << 30])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_split_rows_match_oracle(D, O, split, prec, mode):
    # rows summed in pieces (in-degrees 4095..25000: one to seven pieces)
    # next to rows summed in steps; split = 1: every row in pieces,
    # 1 << 30: none.  Both schemes: in the lock-free one the pieces of a row
    # join the worklist when the row becomes affected
    say("split rows", split, prec, mode)
    n, s, d = inputs.heavy_rows()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 77, frac=1e-3)[0]
    ns, nd, res, ndel, nins = O.update(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m, precision=prec,
               renormalize=int(prec == 32), split_min_degree=split) as g:
        rc, st = g.static()
        assert rc == D.DFPR_OK and st.converged
        Rs = g.ranks()
        g.set_ranks(R0)
        assert g.apply(b) == (ndel, nins)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        R = g.ranks()
    say("  static err", err64(Rs, R0), "update err", err64(R, ref), "iters",
        st.sweeps, "oracle", res.iters)
    if prec == 64:
        assert err64(Rs, R0) < FP64_TOL
        assert err64(R, ref) < FP64_TOL
        if mode == "sync":
            assert abs(st.sweeps - res.iters) <= 1
    else:
        assert rel32(Rs, R0) < FP32_REL
        assert rel32(R, ref) < FP32_REL


def test_sync_update_is_deterministic(D, O):
    # piece sums are added in piece order and every step row is summed by
    # one wavefront, so repeated runs give the same bits; with pieces from
    # in-degree 64 every iteration publishes thousands of partial sums
    # through device-scope stores and counts (a partial read before it
    # landed would change the bits)
    say("determinism")
    n, s, d = inputs.heavy_rows()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 78, frac=1e-2)[0]
    out = []
    for _ in range(4):
        with graph(D, n, s, d, mode=D.DFPR_SYNC, split_min_degree=64) as g:
            g.set_ranks(R0)
            g.apply(b)
            rc, st = g.update()
            assert rc == D.DFPR_OK
            out.append(g.ranks())
    for r in out[1:]:
        assert np.array_equal(out[0], r)


@pytest.mark.parametrize("kind", ["rmat_small", "heavy_rows"])
def test_graph_replay_matches_launches(D, O, kind):
    # the barrier-based loop replayed from a captured HIP graph gives the
    # same bits as launching it iteration by iteration, for several updates
    # in a row on the same graph objects (eager applies between replays, one
    # relocating a hub row; a parameter change forcing a new capture), and
    # static PageRank likewise; both match the oracle
    say("graph replay", kind)
    n, s, d = getattr(inputs, kind)()
    bs = inputs.batches(n, s, d, 3, seed=55, frac=2e-3)
    hub = np.zeros(3000, np.int32) + 7
    grow = inputs.Batch(np.empty(0, np.int32), np.empty(0, np.int32), hub,
                        np.arange(100, 3100, dtype=np.int32))
    cs, cd = s, d
    with graph(D, n, s, d, mode=D.DFPR_SYNC, graph_replay=1) as gr, \
         graph(D, n, s, d, mode=D.DFPR_SYNC, graph_replay=0) as ge:
        for g in (gr, ge):
            rc, st = g.static()
            assert rc == D.DFPR_OK
        assert np.array_equal(gr.ranks(), ge.ranks())
        for k, b in enumerate([bs[0], grow, bs[1], bs[2]]):
            cs, cd, _, _ = O.apply_batch(n, cs, cd, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
            for g in (gr, ge):
                if k == 2:
                    g.set_params(split_min_degree=256)
                g.apply(b)
                rc, st = g.update()
                assert rc == D.DFPR_OK
            Rr, Re = gr.ranks(), ge.ranks()
            assert np.array_equal(Rr, Re), k
        ref, _, _ = O.pagerank(n, cs, cd)
        assert err64(Rr, ref) < FP64_TOL


def test_renormalisation_rescales_drift_only(D, O):
    # fp32 renormalisation: an update whose ranks sum to 1 up to its own
    # truncation (n * tau) is left as it is, bit for bit (the barrier-based
    # scheme is deterministic); ranks that start 0.1% too high everywhere
    # keep that drift on the unaffected vertices, and it is rescaled away
    say("renormalisation")
    n, s, d, R0 = base_graph(O, "rmat_small")
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-3)[0]
    out = {}
    for scale in (1.0, 1.001):
        for renorm in (0, 1):
            with graph(D, n, s, d, mode=D.DFPR_SYNC, precision=32, renormalize=renorm) as g:
                g.set_ranks(R0 * scale)
                g.apply(b)
                rc, st = g.update()
                assert rc == D.DFPR_OK and st.converged
                out[scale, renorm] = g.ranks()
    assert np.array_equal(out[1.0, 0], out[1.0, 1])
    assert abs(out[1.0, 1].sum() - 1.0) < n * 1e-10
    assert abs(out[1.001, 0].sum() - 1.0) > 1e-5
    assert abs(out[1.001, 1].sum() - 1.0) < 1e-6


@pytest.mark.parametrize("mode,kahan", [("sync", 0), ("sync", 8), ("sync", 1 << 30),
                                        ("async", 0)])
def test_df_fp32_matches_oracle(D, O, mode, kahan):
    # kahan_min_degree: rows below it sum in fp32 (barrier-based scheme);
    # 0, the default, sums every row in fp64; 8 splits the 2^14 R-MAT's
    # rows between the two; 2^30 sums every row in fp32
    say("df fp32", mode, kahan)
    n, s, d = inputs.rmat_small()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-3)[0]
    ns, nd, res, _, _ = O.update(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m, precision=32, renormalize=1, kahan_min_degree=kahan) as g:
        g.set_ranks(R0)
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        R = g.ranks()
    say("  rel", rel32(R, ref), "abs", err64(R, ref), "sweeps", st.sweeps)
    assert rel32(R, ref) < FP32_REL


@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("k", [7, 1000, 5000, 20000])
def test_df_star_closed_form(D, O, mode, k):
    say("star", mode, k)
    # out-star -> bidirectional star; the closed forms fix both ends
    a = 0.85
    n = k + 1
    s = np.zeros(k, np.int32)
    d = np.arange(1, n, dtype=np.int32)
    R0 = np.array([(1 - a) / (k + 1 - a)] + [1 / (k + 1 - a)] * k)
    den = (2 - a) + k * (2 + a)
    ref = np.array([((2 - a) + a * k) / den] + [2 / den] * k)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m) as g:
        g.set_ranks(R0)
        ad, ai = g.apply_batch(np.empty(0, np.int32), np.empty(0, np.int32),
                               np.arange(1, n, dtype=np.int32), np.zeros(k, np.int32))
        assert ai == k
        rc, st = g.update()
        assert rc == D.DFPR_OK
        R = g.ranks()
    assert err64(R, ref) < FP64_TOL


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_df_empty_and_noop_batches_keep_ranks(D, O, mode):
    say("empty batch", mode)
    n, s, d = inputs.rmat(10, 8 << 10, seed=4)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m) as g:
        g.static()
        R = g.ranks()
        rc, st = g.update()                     # nothing applied
        assert rc == D.DFPR_OK and st.sweeps == 0
        assert np.array_equal(g.ranks(), R)     # bit-identical
        ad, ai = g.apply_batch(np.array([0], np.int32), np.array([0], np.int32),
                               s[:1], d[:1])    # self pair + existing edge
        assert (ad, ai) == (0, 0)
        assert g.marks()[1] == 0
        rc, st = g.update()
        assert st.sweeps == 0 and np.array_equal(g.ranks(), R)


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_df_sequential_batches_and_stability(D, O, mode):
    say("sequential", mode)
    n, s, d = inputs.rmat_small(seed=5)
    bs = inputs.batches(n, s, d, 3, seed=55, frac=2e-3)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    cs, cd = s, d
    with graph(D, n, s, d, mode=m) as g:
        g.static()
        R_start = g.ranks()
        for b in bs:
            g.apply(b)
            rc, st = g.update()
            assert rc == D.DFPR_OK
            cs, cd, _, _ = O.apply_batch(n, cs, cd, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
            ref, _, _ = O.pagerank(n, cs, cd)
            assert err64(g.ranks(), ref) < FP64_TOL
        # stability round trip (Section 5.2.3): undo every batch in reverse
        for b in reversed(bs):
            g.apply_batch(b.ins_src, b.ins_dst, b.del_src, b.del_dst)
            g.update()
        assert np.array_equal(edge_keys(n, *g.edges()), edge_keys(n, s, d))
        ref0, _, _ = O.pagerank(n, s, d)
        assert err64(g.ranks(), ref0) < FP64_TOL
        assert err64(g.ranks(), R_start) < 2 * FP64_TOL


def test_df_ragged_small_graphs(D, O):
    say("ragged small")
    for seed, (n, m) in enumerate([(1, 0), (2, 1), (63, 200), (65, 300), (129, 2000)]):
        if m:
            _, s, d = inputs.erdos_renyi(n, m, seed=seed)
        else:
            s = d = np.empty(0, np.int32)
        for mode in (D.DFPR_SYNC, D.DFPR_ASYNC):
            with graph(D, n, s, d, mode=mode) as g:
                g.static()
                ref, _, _ = O.pagerank(n, s, d)
                assert err64(g.ranks(), ref) < FP64_TOL
                if n >= 2:
                    b = inputs.Batch(s[:1].copy(), d[:1].copy(),
                                     np.array([n - 1], np.int32), np.array([0], np.int32))
                    ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst,
                                                 b.ins_src, b.ins_dst)
                    g.apply(b)
                    rc, st = g.update()
                    assert rc == D.DFPR_OK
                    ref, _, _ = O.pagerank(n, ns, nd)
                    assert err64(g.ranks(), ref) < FP64_TOL


@pytest.mark.parametrize("kind", ["rmat_small", "heavy_rows"])
@pytest.mark.parametrize("prec", [64, 32])
def test_lock_free_static_and_naive_dynamic(D, O, kind, prec):
    # Algorithms 4 and 6 on the persistent kernel: a full sweep with no
    # change above the frontier tolerance ends the launch, within the
    # paper's cap of 500 sweeps (hub rows are summed in pieces, so no claim
    # holds a whole 25,000-edge row)
    say("lock-free static / ND", kind, prec)
    n, s, d = getattr(inputs, kind)()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 61, frac=1e-2)[0]
    ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
    R1, _, _ = O.pagerank(n, ns, nd)
    with graph(D, n, s, d, mode=D.DFPR_ASYNC, precision=prec,
               renormalize=int(prec == 32)) as g:
        rc, st = g.static_lock_free()
        assert rc == D.DFPR_OK and st.converged and st.affected == n
        Rs = g.ranks()
        g.apply(b)
        rc, st = g.naive_dynamic_lock_free()
        assert rc == D.DFPR_OK and st.converged
        Rn = g.ranks()
        aff, cnt = g.marks()
        assert cnt == 0 and not aff.any()       # the batch counts as served
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.vertices_processed == 0
    say("  static err", err64(Rs, R0), "nd err", err64(Rn, R1))
    if prec == 64:
        assert err64(Rs, R0) < FP64_TOL and err64(Rn, R1) < FP64_TOL
    else:
        assert rel32(Rs, R0) < FP32_REL and rel32(Rn, R1) < FP32_REL


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_injected_faults(D, O, mode):
    # fault simulation: delayed workgroups and workgroups that stop at a
    # claim boundary; the others finish the update, which still matches the
    # oracle; with every workgroup stopped the call fails cleanly
    say("faults", mode)
    n, s, d = inputs.rmat_small()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 1001, frac=1e-3)[0]
    ns, nd, res, _, _ = O.update(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m) as g:
        g.set_ranks(R0)
        g.set_faults([0, -1, 0, 40, -1, 0, 0, -1])   # 3 of 8 stop, 1 delayed
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged
        assert err64(g.ranks(), ref) < FP64_TOL
        if mode == "sync":
            assert abs(st.sweeps - res.iters) <= 1
        # every workgroup stops after one claim: the barrier-based launches
        # still cover every item (a grid has at least as many wavefronts as
        # an iteration of this graph has items, and each is relaunched per
        # iteration); the persistent launch runs out of workers and fails
        g.set_faults([-1])
        ns2, nd2 = ns, nd
        b2 = inputs.batches(n, ns, nd, 1, 1002, frac=1e-3)[0]
        R1 = g.ranks()
        g.apply(b2)
        if mode == "sync":
            ns2, nd2, res2, _, _ = O.update(n, ns, nd, b2, R1)
            rc, st = g.update()
            assert rc == D.DFPR_OK
            ref2, _, _ = O.pagerank(n, ns2, nd2)
            assert err64(g.ranks(), ref2) < FP64_TOL
        else:
            with pytest.raises(D.DfprError) as ei:
                g.update()
            assert ei.value.status == D.DFPR_EABORT
        g.set_faults([])
        with pytest.raises(D.DfprError) as ei:
            g.set_faults([-2])
        assert ei.value.status == D.DFPR_EINVAL


def test_sync_claims_taken_over(D, O):
    # a small grid (8 workgroups of 2 wavefronts) with every fourth
    # workgroup stopping after one claim: the stopped wavefronts' claim
    # counters hold several items each, which the others must take over;
    # with every workgroup stopped the iteration is left incomplete and the
    # call fails cleanly, after which the graph is usable again
    say("sync claims taken over")
    n, s, d = inputs.rmat_small()
    ref, _, _ = O.pagerank(n, s, d)
    with graph(D, n, s, d, mode=D.DFPR_SYNC) as g:
        g.set_params(grid_blocks=8, block_size=128)
        g.set_faults([-1, 0, 0, 0])
        rc, st = g.static()
        assert rc == D.DFPR_OK and st.converged
        assert err64(g.ranks(), ref) < FP64_TOL
        g.set_faults([-1])
        with pytest.raises(D.DfprError) as ei:
            g.static()
        assert ei.value.status == D.DFPR_EABORT
        g.set_faults([])
        rc, st = g.static()
        assert rc == D.DFPR_OK and err64(g.ranks(), ref) < FP64_TOL


@pytest.mark.parametrize("blocks,block", [(1, 64), (3, 128)])
def test_sync_grid_smaller_than_claim_counters(D, O, blocks, block):
    # fewer wavefronts (1 and 6) than claim counters, far fewer than an
    # iteration's work items: every item is still claimed, static and DF
    say("sync tiny grid", blocks, block)
    n, s, d = inputs.rmat_small()
    b = inputs.batches(n, s, d, 1, seed=1301, frac=1e-3)[0]
    R0, _, _ = O.pagerank(n, s, d)
    ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
    ref, _, _ = O.pagerank(n, ns, nd)
    with graph(D, n, s, d, mode=D.DFPR_SYNC) as g:
        g.set_params(grid_blocks=blocks, block_size=block)
        rc, st = g.static()
        assert rc == D.DFPR_OK and st.converged
        assert err64(g.ranks(), R0) < FP64_TOL
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged
        assert err64(g.ranks(), ref) < FP64_TOL


# --- Dynamic Traversal (Algorithms 7 and 8) ------------------------------------

@pytest.mark.parametrize("case", ["sparse_rmat", "grid", "heavy_rows"])
@pytest.mark.parametrize("reorder", [0, 1])
def test_traversal_marks_match_oracle(D, O, case, reorder):
    # the reachable set is unique: compared vertex by vertex; the grid needs
    # ~100 levels (several host polls), the sparse R-MAT leaves part of the
    # graph unreachable, heavy_rows walks out-rows of up to 20000 entries
    say("traversal marks", case, reorder)
    if case == "sparse_rmat":
        n, s, d = inputs.rmat(12, 2 << 12, seed=6)
    elif case == "grid":
        n, s, d = inputs.grid_road(64, 3)
    else:
        n, s, d = inputs.heavy_rows()
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 1003, frac=2e-4)[0]
    ns, nd, res, ndel, nins = O.update_dt(n, s, d, b, R0, max_iters=0)
    with graph(D, n, s, d, reorder=reorder) as g:
        assert g.apply(b) == (ndel, nins)
        cnt = g.mark_reachable()
        aff, cnt2 = g.marks()
        say("  marked", cnt, "oracle", res.initial_marked, "of", n)
        assert cnt == cnt2 == res.initial_marked
        assert np.array_equal(aff.astype(bool), res.affected)
        assert g.mark_reachable() == cnt          # idempotent
    if case == "sparse_rmat":
        assert 0 < cnt < n


@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("prec", [64, 32])
def test_traversal_update_matches_oracle(D, O, mode, prec):
    say("traversal update", mode, prec)
    n, s, d = inputs.rmat(12, 4 << 12, seed=9)
    R0, _, _ = O.pagerank(n, s, d)
    b = inputs.batches(n, s, d, 1, 1004, frac=1e-3)[0]
    ns, nd, res, ndel, nins = O.update_dt(n, s, d, b, R0)
    ref, _, _ = O.pagerank(n, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m, precision=prec,
               renormalize=int(prec == 32)) as g:
        g.set_ranks(R0)
        R0d = g.ranks()                         # R0 as the graph stores it
        assert g.apply(b) == (ndel, nins)
        rc, st = g.update_traversal()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        R = g.ranks()
    say("  sweeps", st.sweeps, "oracle", res.iters, "marked", st.initial_marked,
        res.initial_marked)
    assert st.initial_marked == res.initial_marked
    if prec == 64:
        assert err64(R, ref) < FP64_TOL
        assert err64(R, res.R) < FP64_TOL
        # vertices outside the reachable set are never written
        assert np.array_equal(R[~res.affected], R0d[~res.affected])
    else:
        assert rel32(R, ref) < FP32_REL
    if mode == "sync":
        assert st.affected == res.initial_marked
        assert abs(st.sweeps - res.iters) <= 1


def test_traversal_empty_and_repeat(D, O):
    # nothing marked: no work, ranks bit-identical; a traversal update
    # after a normal DF update starts from fresh marks
    say("traversal empty")
    n, s, d = inputs.rmat_small()
    R0, _, _ = O.pagerank(n, s, d)
    with graph(D, n, s, d) as g:
        g.set_ranks(R0)
        assert g.mark_reachable() == 0
        rc, st = g.update_traversal()
        assert rc == D.DFPR_OK and st.sweeps == 0
        assert np.array_equal(g.ranks(), R0)
        b1, b2 = inputs.batches(n, s, d, 2, 1005, frac=1e-3)
        s1, d1, _, _, _ = O.update(n, s, d, b1, R0)
        g.apply(b1)
        rc, _ = g.update()
        assert rc == D.DFPR_OK
        R1 = g.ranks()
        s2, d2, res2, _, _ = O.update_dt(n, s1, d1, b2, R1)
        ref, _, _ = O.pagerank(n, s2, d2)
        g.apply(b2)
        rc, st = g.update_traversal()
        assert rc == D.DFPR_OK and st.initial_marked == res2.initial_marked
        assert err64(g.ranks(), ref) < FP64_TOL


# --- vertex insertion and removal (rescaled ranks) -------------------------------

@pytest.mark.parametrize("reorder", [0, 1])
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_add_vertices_matches_oracle(D, O, mode, reorder):
    say("add vertices", mode, reorder)
    n, s, d = inputs.rmat_small()
    k = 100
    R0, _, _ = O.pagerank(n, s, d)
    rng = np.random.default_rng(17)
    new = np.arange(n, n + k, dtype=np.int32)
    old = rng.integers(0, n, k).astype(np.int32)
    b = inputs.Batch(np.empty(0, np.int32), np.empty(0, np.int32),
                     np.concatenate([new, old, new[:10]]),
                     np.concatenate([old, new, new[10:20]]))
    ns, nd, res, Rs = O.add_vertices_update(n, s, d, k, b, R0)
    ref, _, _ = O.pagerank(n + k, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m, reorder=reorder) as g:
        g.set_ranks(R0)
        assert g.add_vertices(k) == n
        assert g.size() == (n + k, s.size)
        assert np.array_equal(g.ranks(), Rs)          # same fp64 product
        assert g.marks()[1] == 0
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        assert st.initial_marked == res.initial_marked
        R = g.ranks()
        es, ed = g.edges(D.DFPR_OUT)
    assert np.array_equal(edge_keys(n + k, es, ed), edge_keys(n + k, ns, nd))
    assert err64(R, ref) < FP64_TOL


def test_vertices_fp32(D, O):
    # fp32 ranks: rescaled in fp64 and rounded once; the update after an
    # insertion and a removal lands within the fp32 bar of the oracle
    say("vertices fp32")
    n, s, d = inputs.erdos_renyi(3000, 20000, 6)
    k = 60
    R0, _, _ = O.pagerank(n, s, d)
    rng = np.random.default_rng(23)
    new = np.arange(n, n + k, dtype=np.int32)
    old = rng.integers(0, n, k).astype(np.int32)
    b = inputs.Batch(np.empty(0, np.int32), np.empty(0, np.int32),
                     np.concatenate([new, old]), np.concatenate([old, new]))
    ns, nd, res, Rs = O.add_vertices_update(n, s, d, k, b, R0)
    ref1, _, _ = O.pagerank(n + k, ns, nd)
    ns2, nd2, _, _ = O.remove_vertices_update(n + k, ns, nd, 2 * k, ref1)
    ref2, _, _ = O.pagerank(n - k, ns2, nd2)
    with graph(D, n, s, d, precision=32, renormalize=1) as g:
        g.set_ranks(R0)
        g.add_vertices(k)
        assert rel32(g.ranks(), Rs) < 3e-7          # two fp32 roundings
        g.apply(b)
        rc, st = g.update()
        assert rc == D.DFPR_OK and rel32(g.ranks(), ref1) < FP32_REL
        g.remove_vertices(2 * k)
        rc, st = g.update()
        assert rc == D.DFPR_OK and rel32(g.ranks(), ref2) < FP32_REL


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_remove_vertices_matches_oracle(D, O, mode):
    say("remove vertices", mode)
    n, s, d = inputs.erdos_renyi(3000, 20000, 5)
    k = 120
    R0, _, _ = O.pagerank(n, s, d)
    _, _, res0, Rs = O.remove_vertices_update(n, s, d, k, R0, max_iters=0)
    ns, nd, res, _ = O.remove_vertices_update(n, s, d, k, R0)
    ref, _, _ = O.pagerank(n - k, ns, nd)
    m = D.DFPR_SYNC if mode == "sync" else D.DFPR_ASYNC
    with graph(D, n, s, d, mode=m) as g:
        g.set_ranks(R0)
        g.remove_vertices(k)
        assert g.size() == (n - k, ns.size)
        assert np.array_equal(g.ranks(), Rs)
        aff, cnt = g.marks()
        assert cnt == res0.initial_marked
        assert np.array_equal(aff, res0.affected)
        rc, st = g.update()
        assert rc == D.DFPR_OK and st.converged, st.as_dict()
        R = g.ranks()
        es, ed = g.edges(D.DFPR_OUT)
    assert np.array_equal(edge_keys(n - k, es, ed), edge_keys(n - k, ns, nd))
    assert err64(R, ref) < FP64_TOL


def test_vertices_round_trip_and_errors(D, O):
    say("vertices round trip")
    n, s, d = inputs.rmat_small()
    # hubs at the highest ids: a degree-sorted graph moves them inside
    s, d = (n - 1 - s).astype(np.int32), (n - 1 - d).astype(np.int32)
    R0, _, _ = O.pagerank(n, s, d)
    with graph(D, n, s, d, reorder=1) as g:
        g.set_ranks(R0)
        with pytest.raises(D.DfprError) as ei:
            g.remove_vertices(3)
        assert ei.value.status == D.DFPR_EINVAL
        for bad in (0, n):
            with pytest.raises(D.DfprError):
                g.remove_vertices(bad)
        with pytest.raises(D.DfprError):
            g.add_vertices(0)
        assert g.add_vertices(7) == n
        g.remove_vertices(7)                  # added vertices keep their ids
        assert g.size() == (n, s.size)
        assert float(np.abs(g.ranks() - R0).max()) < 1e-15
        rc, st = g.update()                   # nothing was marked
        assert rc == D.DFPR_OK and st.sweeps == 0
        es, ed = g.edges(D.DFPR_OUT)
        assert np.array_equal(edge_keys(n, es, ed), edge_keys(n, s, d))


def test_naive_dynamic_matches_oracle(D, O):
    say("naive dynamic")
    n, s, d = inputs.rmat_small()
    b = inputs.batches(n, s, d, 1, 7, frac=1e-2)[0]
    ns, nd, _, _ = O.apply_batch(n, s, d, b.del_src, b.del_dst, b.ins_src, b.ins_dst)
    ref, _, _ = O.pagerank(n, ns, nd)
    with graph(D, n, s, d) as g:
        g.static()
        g.apply(b)
        rc, st = g.naive_dynamic()
        assert rc == D.DFPR_OK
        assert err64(g.ranks(), ref) < FP64_TOL
