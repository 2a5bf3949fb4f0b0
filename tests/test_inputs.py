"""Properties of the seeded synthetic inputs shared by the oracle and the HIP
path: exact sizes, no self pairs or duplicates, batches that are true
changes, and the exact hub degrees of the heavy-row graph."""
import numpy as np
import pytest

from paper_2407_19562_amd import inputs


def keys(n, s, d):
    return s.astype(np.int64) * n + d


@pytest.mark.parametrize("scale,m,seed", [(8, 1000, 3), (12, 8 << 12, 1), (14, 8 << 14, 1)])
def test_rmat_exact_simple(scale, m, seed):
    n, s, d = inputs.rmat(scale, m, seed)
    assert n == 1 << scale and s.size == m and d.size == m
    assert s.dtype == np.int32 and d.dtype == np.int32
    assert (s != d).all()
    assert np.unique(keys(n, s, d)).size == m
    assert s.min() >= 0 and max(s.max(), d.max()) < n


def test_rmat_is_deterministic_and_skewed():
    a = inputs.rmat(12, 8 << 12, 5)
    b = inputs.rmat(12, 8 << 12, 5)
    assert all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))
    n, s, d = a
    indeg = np.bincount(d, minlength=n)
    # power law: the top 1% of vertices hold far more than 1% of the edges
    top = np.sort(indeg)[-n // 100:].sum()
    assert top > 0.05 * s.size


def test_erdos_renyi_exact_simple():
    n, s, d = inputs.erdos_renyi(500, 3000, 9)
    assert n == 500 and s.size == 3000 and (s != d).all()
    assert np.unique(keys(n, s, d)).size == 3000


def test_grid_road_small():
    n, s, d = inputs.grid_road(64, 3)
    assert n == 64 * 64 and (s != d).all()
    assert np.unique(keys(n, s, d)).size == s.size
    outdeg = np.bincount(s, minlength=n)
    assert outdeg.max() <= 5


@pytest.mark.parametrize("frac", [1e-3, 5e-2])
def test_batches_are_true_changes(frac):
    n, s, d = inputs.rmat(12, 8 << 12, 1)
    existing = set(keys(n, s, d).tolist())
    bs = inputs.batches(n, s, d, 3, seed=11, frac=frac)
    total = inputs.batch_counts(s.size, frac=frac)
    dels, inss = [], []
    for b in bs:
        assert b.del_src.size + b.ins_src.size == sum(total)
        dk = keys(n, b.del_src, b.del_dst)
        ik = keys(n, b.ins_src, b.ins_dst)
        assert all(k in existing for k in dk.tolist())
        assert not any(k in existing for k in ik.tolist())
        assert (b.ins_src != b.ins_dst).all()
        dels.extend(dk.tolist())
        inss.extend(ik.tolist())
    # batches drawn together stay distinct, so they apply in sequence
    assert len(set(dels)) == len(dels) and len(set(inss)) == len(inss)


def test_batch_shares_are_80_20():
    nd, ni = inputs.batch_counts(100000, frac=1e-2)
    assert nd + ni == 1000 and ni == 800


def test_heavy_rows_exact_hubs():
    n, s, d = inputs.heavy_rows()
    indeg = np.bincount(d, minlength=n)
    outdeg = np.bincount(s, minlength=n)
    assert indeg[:6].tolist() == [4095, 4096, 4097, 8192, 12289, 25000]
    assert outdeg[6:9].tolist() == [4096, 9000, 20000]
    assert (s != d).all() and np.unique(keys(n, s, d)).size == s.size


def test_graph_mix_sizes():
    mix = list(inputs.graph_mix(16, 77, m_lo=200, m_hi=20000))
    assert len(mix) == 16
    kinds = {k for k, _, _, _ in mix}
    assert kinds <= {"rmat", "er"}
    for kind, n, s, d in mix:
        assert s.size == d.size and s.size >= 1
        assert (s != d).all() and max(s.max(), d.max()) < n
