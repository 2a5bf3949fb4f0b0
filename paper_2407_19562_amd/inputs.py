"""Seeded synthetic inputs: graphs and edge-update batches.

This module holds no PageRank arithmetic and applies no batch: it only draws
edge lists.  Both the HIP path (tests, bench, serving driver) and the CPU
oracle read the arrays it returns, so the two sides always see the same input.

The paper measures on SNAP temporal graphs and SuiteSparse web, social, road
and k-mer graphs (Section 5.1.3, Tables 1 and 2).  None of them is available
here, so these generators stand in for them:

* ``rmat``  -- power-law directed graphs (web/social class), R-MAT recursion
  with quadrant probabilities (a, b, c, d), self pairs and duplicates dropped,
  then a seeded random relabelling of vertices so that ids carry no locality.
* ``erdos_renyi`` -- G(n, m) uniform directed graphs.
* ``grid_road`` -- high-diameter road-like graph: a 2D grid with bidirectional
  4-neighbour edges, a fraction of undirected pairs removed, plus a few random
  long-range edges from distinct sources (out-degree stays <= 5).
* ``batches`` -- update batches following Section 5.1.4: deletions are
  existing edges chosen uniformly, insertions are uniformly chosen vertex pairs
  that are not connected (and not self pairs).  Several batches are drawn at
  once so that, applied one after the other, every deletion still names a
  present edge and every insertion an absent one.

Every function returns int32 numpy arrays ``(src, dst)``; vertex ids are in
``[0, n)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _unique_first(keys: np.ndarray) -> np.ndarray:
    """Distinct keys, kept in order of first appearance (seed-stable)."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return keys[first]


def _sorted_unique(keys: np.ndarray) -> np.ndarray:
    """Distinct values of ``keys`` in increasing order (sorts in place)."""
    keys.sort()
    if keys.size == 0:
        return keys
    keep = np.empty(keys.size, dtype=bool)
    keep[0] = True
    np.not_equal(keys[1:], keys[:-1], out=keep[1:])
    return keys[keep]


# Quadrant probabilities are applied at 16-bit resolution: one uniform
# 16-bit integer per recursion level picks the quadrant.
_Q = 65536


def _rmat_keys(rng, count: int, scale: int, n: int, a: float, b: float,
               c: float, chunk: int = 1 << 20) -> np.ndarray:
    """``count`` R-MAT samples as keys src*n+dst; self pairs and ids >= n
    are returned as -1."""
    t1 = int(round(a * _Q))
    t2 = int(round((a + b) * _Q))
    t3 = int(round((a + b + c) * _Q))
    out = np.empty(count, dtype=np.int64)
    for s0 in range(0, count, chunk):
        k = min(chunk, count - s0)
        u = rng.integers(0, _Q, (scale, k), dtype=np.uint16)
        src = np.zeros(k, dtype=np.int64)
        dst = np.zeros(k, dtype=np.int64)
        for lvl in range(scale):
            ul = u[lvl]
            right = ul >= t2                     # lower half: c or d quadrant
            down = (ul >= t1) ^ right ^ (ul >= t3)  # b or d quadrant
            src <<= 1
            src |= right
            dst <<= 1
            dst |= down
        key = src * n + dst
        key[(src == dst) | (src >= n) | (dst >= n)] = -1
        out[s0:s0 + k] = key
    return out


def rmat(scale: int, m: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, n: int | None = None, permute: bool = True):
    """R-MAT digraph with exactly ``m`` distinct non-self edges.

    Quadrant recursion over ``scale`` levels with probabilities (a, b, c,
    1-a-b-c) and no noise; self pairs and duplicates are dropped and more
    samples are drawn until ``m`` distinct edges exist, surplus edges are
    dropped uniformly at random, then vertices are relabelled by a seeded
    random permutation.  ``n`` defaults to ``2**scale``; a smaller ``n``
    rejects sampled ids >= n (vertex counts that are not powers of two).
    """
    if n is None:
        n = 1 << scale
    if n > (1 << scale):
        raise ValueError("n exceeds 2**scale")
    if m > n * (n - 1):
        raise ValueError("too many edges for n")
    rng = np.random.default_rng(seed)
    keys = np.empty(0, dtype=np.int64)
    want = int(m * 1.05) + 1024
    while True:
        fresh = _rmat_keys(rng, want, scale, n, a, b, c)
        keys = _sorted_unique(np.concatenate([keys, fresh[fresh >= 0]]))
        del fresh
        if keys.size >= m:
            break
        want = int((m - keys.size) * 1.5) + 1024
    if keys.size > m:
        drop = rng.choice(keys.size, keys.size - m, replace=False)
        keys = np.delete(keys, drop)
    src = keys // n
    dst = keys - src * n
    del keys
    if permute:
        perm = rng.permutation(n)
        src = perm[src]
        dst = perm[dst]
    return n, src.astype(np.int32), dst.astype(np.int32)


def erdos_renyi(n: int, m: int, seed: int):
    """Uniform G(n, m) digraph: ``m`` distinct non-self ordered pairs."""
    if m > n * (n - 1):
        raise ValueError("too many edges for n")
    rng = np.random.default_rng(seed)
    have = np.empty(0, dtype=np.int64)
    want = m
    while have.size < m:
        draw = int(want * 1.1) + 64
        s = rng.integers(0, n, draw, dtype=np.int64)
        d = rng.integers(0, n, draw, dtype=np.int64)
        ok = s != d
        have = _unique_first(np.concatenate([have, s[ok] * n + d[ok]]))
        want = max(m - have.size, 1) * 2
    have = have[:m]
    return n, (have // n).astype(np.int32), (have % n).astype(np.int32)


def grid_road(side: int, seed: int, remove_frac: float = 0.05,
              long_range_frac: float = 1e-4):
    """Road-like grid: bidirectional 4-neighbour lattice on side x side
    vertices, ``remove_frac`` of the undirected pairs removed (both
    directions), then ``round(long_range_frac * |E|)`` directed long-range
    edges from distinct sources to uniform targets."""
    rng = np.random.default_rng(seed)
    n = side * side
    ids = np.arange(n, dtype=np.int64).reshape(side, side)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    pu = np.concatenate([hu, vu])
    pv = np.concatenate([hv, vv])
    npairs = pu.size
    n_remove = int(round(remove_frac * npairs))
    keep = np.ones(npairs, dtype=bool)
    keep[rng.choice(npairs, n_remove, replace=False)] = False
    pu, pv = pu[keep], pv[keep]
    src = np.concatenate([pu, pv])
    dst = np.concatenate([pv, pu])
    m0 = src.size
    n_long = int(round(long_range_frac * m0))
    existing = np.sort(src * n + dst)
    srcs = rng.choice(n, n_long, replace=False).astype(np.int64)
    tgt = np.empty(n_long, dtype=np.int64)
    todo = np.arange(n_long)
    while todo.size:
        t = rng.integers(0, n, todo.size, dtype=np.int64)
        k = srcs[todo] * n + t
        pos = np.searchsorted(existing, k)
        pos[pos >= existing.size] = existing.size - 1
        bad = (t == srcs[todo]) | (existing[pos] == k)
        tgt[todo[~bad]] = t[~bad]
        todo = todo[bad]
    src = np.concatenate([src, srcs])
    dst = np.concatenate([dst, tgt])
    return n, src.astype(np.int32), dst.astype(np.int32)


@dataclass
class Batch:
    """One update batch: deletions (del_src, del_dst) and insertions
    (ins_src, ins_dst), int32 arrays."""
    del_src: np.ndarray
    del_dst: np.ndarray
    ins_src: np.ndarray
    ins_dst: np.ndarray

    @property
    def size(self) -> int:
        return int(self.del_src.size + self.ins_src.size)


def batch_counts(num_edges: int, frac: float | None = None,
                 size: int | None = None, ins_share: float = 0.8):
    """Sizes (n_del, n_ins) of a batch of ``round(frac*|E|)`` (or ``size``)
    edges with an ``ins_share`` fraction of insertions."""
    if size is None:
        size = max(1, int(round(frac * num_edges)))
    n_ins = int(round(ins_share * size))
    return size - n_ins, n_ins


def batches(n: int, src: np.ndarray, dst: np.ndarray, count: int, seed: int,
            frac: float | None = None, size: int | None = None,
            ins_share: float = 0.8) -> list[Batch]:
    """``count`` batches to be applied one after the other to the graph
    (src, dst).  Deletions across all batches are distinct existing edges;
    insertions across all batches are distinct non-edges (u != v) of the
    base graph, so every batch stays a true change of the evolving graph."""
    rng = np.random.default_rng(seed)
    m = src.size
    n_del, n_ins = batch_counts(m, frac, size, ins_share)
    if count * n_del > m:
        raise ValueError("not enough edges to delete")
    pick = rng.choice(m, count * n_del, replace=False) if n_del else \
        np.empty(0, dtype=np.int64)
    ds, dd = src[pick].astype(np.int32), dst[pick].astype(np.int32)
    existing = np.sort(src.astype(np.int64) * n + dst.astype(np.int64))
    need = count * n_ins
    got = np.empty(0, dtype=np.int64)
    while got.size < need:
        draw = int((need - got.size) * 1.1) + 16
        u = rng.integers(0, n, draw, dtype=np.int64)
        v = rng.integers(0, n, draw, dtype=np.int64)
        k = u * n + v
        k = _sorted_unique(np.concatenate([got, k[u != v]]))
        if existing.size:
            pos = np.searchsorted(existing, k)
            pos[pos >= existing.size] = existing.size - 1
            k = k[existing[pos] != k]
        got = k
    got = got[rng.permutation(got.size)[:need]]
    is_, id_ = (got // n).astype(np.int32), (got % n).astype(np.int32)
    out = []
    for i in range(count):
        out.append(Batch(ds[i * n_del:(i + 1) * n_del].copy(),
                         dd[i * n_del:(i + 1) * n_del].copy(),
                         is_[i * n_ins:(i + 1) * n_ins].copy(),
                         id_[i * n_ins:(i + 1) * n_ins].copy()))
    return out


def log_uniform(rng: np.random.Generator, lo: float, hi: float, size=None):
    """Samples whose logarithm is uniform on [log lo, log hi]."""
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


# --- named workloads ---------------------------------------------------------

def rmat_small(seed: int = 1):
    """R-MAT with 2^14 vertices and 131,072 edges (a=.57, b=c=.19)."""
    return rmat(14, 8 << 14, seed)


def rmat_mid(seed: int = 7):
    """R-MAT with 2^20 vertices and average degree 4 (4,194,304 edges): the
    smallest size at which the library switches to its large-graph paths
    (1024-vertex tiles, degree-sorted vertex order)."""
    return rmat(20, 4 << 20, seed)


def rmat_large(seed: int = 2):
    """R-MAT with 2^22 vertices and 16*2^22 = 67,108,864 edges."""
    return rmat(22, 16 << 22, seed)


def road_grid(seed: int = 3, side: int = 4096):
    """4096 x 4096 road-like grid (about 63.7M directed edges)."""
    return grid_road(side, seed)


def heavy_rows(seed: int = 5, n: int = 30000, avg_degree: int = 4,
               hub_in=(4095, 4096, 4097, 8192, 12289, 25000),
               hub_out=(4096, 9000, 20000)):
    """G(n, m) with average degree `avg_degree`, plus in-hubs
    0..len(hub_in)-1 whose in-degrees are exactly the listed values (edges
    from distinct random sources; rows just below, at and above 4096 and
    several times that) and out-hubs numbered after them whose out-degrees
    are exactly `hub_out`.  Returns (n, src, dst) without duplicates."""
    rng = np.random.default_rng(seed)
    n0, s0, d0 = erdos_renyi(n, n * avg_degree, seed)
    h_in = len(hub_in)
    outs = np.arange(h_in, h_in + len(hub_out))
    keep = (d0 >= h_in) & ~np.isin(s0, outs)   # hubs get only the edges below
    keys = [s0[keep].astype(np.int64) * n + d0[keep]]
    for h, k in enumerate(hub_in):
        src = rng.choice(n, size=k + 1 + len(outs), replace=False)
        src = src[(src != h) & ~np.isin(src, outs)][:k]
        keys.append(src.astype(np.int64) * n + h)
    for h, k in zip(outs, hub_out):
        dst = rng.choice(np.arange(h_in, n), size=k + 1, replace=False)
        dst = dst[dst != h][:k]
        keys.append(np.int64(h) * n + dst.astype(np.int64))
    keys = np.unique(np.concatenate(keys))
    keys = rng.permutation(keys)
    return n, (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def graph_mix(count: int, seed: int, m_lo: float = 1e3, m_hi: float = 1e6,
              deg_lo: float = 4, deg_hi: float = 32):
    """Many small graphs: edge counts log-uniform in [m_lo, m_hi], average
    degree log-uniform in [deg_lo, deg_hi], half R-MAT and half G(n, m).
    Yields (kind, n, src, dst) per graph; graph g uses seed ``seed + g``."""
    rng = np.random.default_rng(seed)
    ms = log_uniform(rng, m_lo, m_hi, count)
    degs = log_uniform(rng, deg_lo, deg_hi, count)
    kinds = rng.integers(0, 2, count)
    for g in range(count):
        m = int(round(ms[g]))
        n = max(8, int(round(m / degs[g])))
        m = min(m, n * (n - 1) // 2)
        if kinds[g] == 0:
            scale = max(1, math.ceil(math.log2(n)))
            yield ("rmat",) + rmat(scale, m, seed + 1 + g, n=n)
        else:
            yield ("er",) + erdos_renyi(n, m, seed + 1 + g)


def resident_mix(count: int, seed: int, n_lo: int = 1 << 16,
                 n_hi: int = 1 << 21, deg_lo: float = 8, deg_hi: float = 32):
    """Resident graphs for serving: R-MAT, n log-uniform in [n_lo, n_hi],
    average degree log-uniform in [deg_lo, deg_hi]; graph g uses seed
    ``seed + g``.  Yields (n, src, dst)."""
    rng = np.random.default_rng(seed)
    ns = log_uniform(rng, n_lo, n_hi, count)
    degs = log_uniform(rng, deg_lo, deg_hi, count)
    for g in range(count):
        n = int(round(ns[g]))
        m = int(round(n * degs[g]))
        scale = math.ceil(math.log2(n))
        yield rmat(scale, m, seed + 1 + g, n=n)


# --- on-disk cache of generated inputs (same process tree / same box) ---------

def cached(name: str, fn, *args, **kw):
    """Returns fn(*args, **kw), memoised as an .npz under $DFPR_CACHE_DIR
    (default: $TMPDIR/dfpr_inputs) so that several runs on one machine draw
    the large graphs once.  The key is the name and the arguments."""
    import hashlib
    import os
    import tempfile
    root = os.environ.get("DFPR_CACHE_DIR",
                          os.path.join(tempfile.gettempdir(), "dfpr_inputs"))
    key = hashlib.sha1(repr((name, args, sorted(kw.items()))).encode()).hexdigest()[:16]
    path = os.path.join(root, f"{name}_{key}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return int(z["n"]), z["src"], z["dst"]
    n, src, dst = fn(*args, **kw)
    try:
        os.makedirs(root, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, n=np.int64(n), src=src, dst=dst)
        os.replace(tmp, path)
    except OSError:
        pass
    return n, src, dst
