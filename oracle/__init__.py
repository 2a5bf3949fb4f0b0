"""CPU oracle for Dynamic Frontier PageRank -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The HIP library never uses it,
and nothing here imports the library: the two share only the seeded input
generators.

Layers:
* set operations on edge lists, in numpy (the batch model of Section 3.4:
  E^t = (E^{t-1} minus the deletions) union the insertions, vertex set fixed);
* self-loops on every vertex (dead-end removal, Section 5.1.3);
* fp64 iteration in plain C (``dfpr_oracle.c``): static PageRank of Eq. 1 /
  Algorithm 3, barrier-based Dynamic Frontier of Algorithm 1, and
  barrier-based Dynamic Traversal of Algorithm 7;
* vertex insertion and removal with rescaled ranks before DF (the paper's
  future-work remark), in numpy around the DF iteration.

Readings taken where the paper is silent are listed in the design notes:
self pairs in a batch are ignored (every vertex keeps its self-loop),
inserting an existing edge or deleting an absent one changes nothing and
marks nothing, and a vertex marked during a DF iteration is first
recomputed in the next iteration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfpr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ALPHA = 0.85          # damping factor (Section 5.1.2)
TOL = 1e-10           # iteration tolerance, L-infinity (Section 5.1.2)
FTOL = TOL / 1000     # frontier tolerance (Section 4.4)
MAX_ITERS = 500       # iteration cap (Section 5.1.2)
L1_TOL = 1e-13        # oracle's own stop: L1 change of one sweep


def build() -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        p = ctypes.c_void_p
        lib.oracle_pagerank.argtypes = [i32, i64, p, p, dbl, dbl, i32, i32, p,
                                        p, p, p, p]
        lib.oracle_sweeps.argtypes = [i32, i64, p, p, dbl, i32, i32, p, p, p]
        lib.oracle_df_bb.argtypes = [i32, i64, p, p, i64, p, p, i64, p, p, p,
                                     dbl, dbl, dbl, i32, p, p, p, p, p, p, p]
        lib.oracle_dt_bb.argtypes = [i32, i64, p, p, i64, p, p, i64, p, p,
                                     dbl, dbl, i32, p, p, p, p, p, p, p]
        lib.oracle_residual.argtypes = [i32, i64, p, p, dbl, p, i32, p, p]
        lib.oracle_num_threads.restype = i32
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


# --- edge-set operations (Section 3.4) ---------------------------------------

def keys_of(n: int, src, dst) -> np.ndarray:
    return np.asarray(src, np.int64) * n + np.asarray(dst, np.int64)


def split_keys(n: int, keys: np.ndarray):
    keys = np.asarray(keys, np.int64)
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def edge_set(n: int, src, dst) -> np.ndarray:
    """Sorted distinct keys u*n+v of the pairs, self pairs dropped."""
    k = keys_of(n, src, dst)
    k = k[(k // n) != (k % n)]
    return np.unique(k)


def apply_batch(n: int, src, dst, del_src, del_dst, ins_src, ins_dst):
    """E^t = (E^{t-1} \\ D) U I with set semantics (deletions first).

    Returns (src, dst) of E^t without self pairs, and the true changes
    Delta- = E^{t-1} n D and Delta+ = I \\ (E^{t-1} \\ D) as sorted keys.
    """
    e = edge_set(n, src, dst)
    d = edge_set(n, del_src, del_dst)
    i = edge_set(n, ins_src, ins_dst)
    d_true = np.intersect1d(e, d, assume_unique=True)
    kept = np.setdiff1d(e, d_true, assume_unique=True)
    i_true = np.setdiff1d(i, kept, assume_unique=True)
    new = np.union1d(kept, i_true)
    s, t = split_keys(n, new)
    return s, t, d_true, i_true


def with_self_loops(n: int, src, dst):
    """Adds (v, v) for every vertex (dead-end removal, Section 5.1.3)."""
    k = edge_set(n, src, dst)
    s, t = split_keys(n, k)
    v = np.arange(n, dtype=np.int32)
    return np.concatenate([s, v]), np.concatenate([t, v])


# --- iteration (C) ------------------------------------------------------------

def pagerank(n: int, src, dst, alpha: float = ALPHA, l1_tol: float = L1_TOL,
             max_iters: int = MAX_ITERS, threads: int = 0, init=None,
             self_loops: bool = True):
    """Static PageRank (Eq. 1, Algorithm 3) as the fixed point to fp64
    rounding: Jacobi sweeps from 1/n until the L1 change <= l1_tol.
    Returns (R, iters, last_l1_change)."""
    if self_loops:
        s, t = with_self_loops(n, src, dst)
    else:
        k = np.unique(keys_of(n, src, dst))
        s, t = split_keys(n, k)
    s = np.ascontiguousarray(s, np.int32)
    t = np.ascontiguousarray(t, np.int32)
    R = np.empty(n, np.float64)
    it = ctypes.c_int32()
    l1 = ctypes.c_double()
    linf = ctypes.c_double()
    ini = None if init is None else np.ascontiguousarray(init, np.float64)
    rc = _lib().oracle_pagerank(n, s.size, _ptr(s), _ptr(t), alpha, l1_tol,
                                max_iters, threads, _ptr(ini), _ptr(R),
                                ctypes.byref(it), ctypes.byref(l1),
                                ctypes.byref(linf))
    if rc != 0:
        raise ValueError(f"oracle_pagerank failed ({rc})")
    return R, it.value, l1.value


def residual(n: int, src, dst, R, alpha: float = ALPHA, threads: int = 0,
             self_loops: bool = True):
    """(max_v |T(R)[v]-R[v]|, sum_v |T(R)[v]-R[v]|) for Eq. 1's map T."""
    if self_loops:
        s, t = with_self_loops(n, src, dst)
    else:
        s, t = np.asarray(src, np.int32), np.asarray(dst, np.int32)
    s = np.ascontiguousarray(s, np.int32)
    t = np.ascontiguousarray(t, np.int32)
    R = np.ascontiguousarray(R, np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    rc = _lib().oracle_residual(n, s.size, _ptr(s), _ptr(t), alpha, _ptr(R),
                                threads, ctypes.byref(a), ctypes.byref(b))
    if rc != 0:
        raise ValueError(f"oracle_residual failed ({rc})")
    return a.value, b.value


def timed_sweeps(n: int, src, dst, sweeps: int, threads: int = 0,
                 alpha: float = ALPHA):
    """Runs exactly ``sweeps`` Jacobi sweeps of Eq. 1 (with self-loops).
    Returns (edges_per_sweep, sweep_seconds, build_seconds)."""
    s, t = with_self_loops(n, src, dst)
    s = np.ascontiguousarray(s, np.int32)
    t = np.ascontiguousarray(t, np.int32)
    R = np.empty(n, np.float64)
    b, w = ctypes.c_double(), ctypes.c_double()
    rc = _lib().oracle_sweeps(n, s.size, _ptr(s), _ptr(t), alpha, sweeps,
                              threads, _ptr(R), ctypes.byref(b),
                              ctypes.byref(w))
    if rc != 0:
        raise ValueError(f"oracle_sweeps failed ({rc})")
    return int(s.size), w.value, b.value


class DFResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def df_bb(n: int, prev, cur, sources, R_prev, alpha: float = ALPHA,
          tol: float = TOL, ftol: float = FTOL, max_iters: int = MAX_ITERS,
          self_loops: bool = True, marks=None) -> DFResult:
    """Dynamic Frontier, barrier-based (Algorithm 1) from R_prev.

    ``prev`` and ``cur`` are (src, dst) of G^{t-1} and G^t, ``sources`` the
    u of every true change (u, v) of the batch.  With ``self_loops`` both
    graphs get (v, v) on every vertex first.  ``marks`` (bool[n], optional)
    adds initial marks made outside the two edge sets."""
    ps, pt, cs, ct = _prepared(n, prev, cur, self_loops)
    b = np.ascontiguousarray(sources, np.int32)
    Rp = np.ascontiguousarray(R_prev, np.float64)
    R = np.empty(n, np.float64)
    aff = np.empty(n, np.uint8)
    it = ctypes.c_int32()
    dR = ctypes.c_double()
    im, wv, we = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    m0 = None if marks is None else np.ascontiguousarray(marks, np.uint8)
    rc = _lib().oracle_df_bb(n, ps.size, _ptr(ps), _ptr(pt), cs.size,
                             _ptr(cs), _ptr(ct), b.size, _ptr(b), _ptr(m0),
                             _ptr(Rp),
                             alpha, tol, ftol, max_iters, _ptr(R), _ptr(aff),
                             ctypes.byref(it), ctypes.byref(dR),
                             ctypes.byref(im), ctypes.byref(wv),
                             ctypes.byref(we))
    if rc != 0:
        raise ValueError(f"oracle_df_bb failed ({rc})")
    return DFResult(R=R, affected=aff.astype(bool), iters=it.value,
                    last_dR=dR.value, initial_marked=im.value,
                    work_vertices=wv.value, work_edges=we.value)


def _prepared(n, prev, cur, self_loops):
    if self_loops:
        ps, pt = with_self_loops(n, *prev)
        cs, ct = with_self_loops(n, *cur)
    else:
        ps, pt = split_keys(n, edge_set(n, *prev))
        cs, ct = split_keys(n, edge_set(n, *cur))
    return tuple(np.ascontiguousarray(a, np.int32) for a in (ps, pt, cs, ct))


def dt_bb(n: int, prev, cur, sources, R_prev, alpha: float = ALPHA,
          tol: float = TOL, max_iters: int = MAX_ITERS,
          self_loops: bool = True) -> DFResult:
    """Dynamic Traversal, barrier-based (Algorithm 7) from R_prev: every
    vertex reachable in G^t from the previous or current out-neighbours of
    a batch source is affected, then Jacobi sweeps over that fixed set.
    Arguments as for df_bb; ``initial_marked`` is the affected count."""
    ps, pt, cs, ct = _prepared(n, prev, cur, self_loops)
    b = np.ascontiguousarray(sources, np.int32)
    Rp = np.ascontiguousarray(R_prev, np.float64)
    R = np.empty(n, np.float64)
    aff = np.empty(n, np.uint8)
    it = ctypes.c_int32()
    dR = ctypes.c_double()
    im, wv, we = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = _lib().oracle_dt_bb(n, ps.size, _ptr(ps), _ptr(pt), cs.size,
                             _ptr(cs), _ptr(ct), b.size, _ptr(b), _ptr(Rp),
                             alpha, tol, max_iters, _ptr(R), _ptr(aff),
                             ctypes.byref(it), ctypes.byref(dR),
                             ctypes.byref(im), ctypes.byref(wv),
                             ctypes.byref(we))
    if rc != 0:
        raise ValueError(f"oracle_dt_bb failed ({rc})")
    return DFResult(R=R, affected=aff.astype(bool), iters=it.value,
                    last_dR=dR.value, initial_marked=im.value,
                    work_vertices=wv.value, work_edges=we.value)


def update_dt(n: int, src, dst, batch, R_prev, **kw):
    """As update, with dt_bb in place of df_bb."""
    s, t, d_true, i_true = apply_batch(n, src, dst, batch.del_src,
                                       batch.del_dst, batch.ins_src,
                                       batch.ins_dst)
    sources = np.concatenate([d_true // n, i_true // n]).astype(np.int32)
    res = dt_bb(n, (src, dst), (s, t), sources, R_prev, **kw)
    return s, t, res, int(d_true.size), int(i_true.size)


def update(n: int, src, dst, batch, R_prev, **kw):
    """Applies ``batch`` (an inputs.Batch) to (src, dst) and runs df_bb.
    Returns (new_src, new_dst, DFResult, n_deleted, n_inserted)."""
    s, t, d_true, i_true = apply_batch(n, src, dst, batch.del_src,
                                       batch.del_dst, batch.ins_src,
                                       batch.ins_dst)
    sources = np.concatenate([d_true // n, i_true // n]).astype(np.int32)
    res = df_bb(n, (src, dst), (s, t), sources, R_prev, **kw)
    return s, t, res, int(d_true.size), int(i_true.size)


# --- vertex insertion and removal ---------------------------------------------
#
# The paper fixes the vertex set (Section 3.4) and names vertex additions
# and deletions, with the existing ranks scaled before the computation, as
# future work (Section 6).  Reading: Eq. 1's teleport term is (1-alpha)/n,
# so multiplying a fixed point by n_old/n_new gives a fixed point for the
# new term wherever the edges did not change; an added vertex starts at
# 1/n_new, the rank of an isolated vertex with its self-loop.  Added
# vertices take the next ids; removal takes the highest ids, with every
# incident edge.

def rescale(R_prev, n_new: int) -> np.ndarray:
    """Ranks for a vertex count changed from R_prev.size to n_new: kept
    vertices times n_old / n_new, added vertices at 1 / n_new."""
    R_prev = np.asarray(R_prev, np.float64)
    n_old = R_prev.size
    f = float(n_old) / float(n_new)
    keep = min(n_old, n_new)
    R = np.full(n_new, 1.0 / n_new)
    R[:keep] = R_prev[:keep] * f
    return R


def add_vertices_update(n: int, src, dst, k: int, batch, R_prev, **kw):
    """k isolated vertices appended (ids n .. n+k-1), ranks rescaled, then
    ``batch`` applied on the n+k vertices and DF run from the rescaled
    ranks.  Returns (new_src, new_dst, DFResult, rescaled ranks)."""
    n1 = n + k
    R = rescale(R_prev, n1)
    s, t, d_true, i_true = apply_batch(n1, src, dst, batch.del_src,
                                       batch.del_dst, batch.ins_src,
                                       batch.ins_dst)
    sources = np.concatenate([d_true // n1, i_true // n1]).astype(np.int32)
    res = df_bb(n1, (src, dst), (s, t), sources, R, **kw)
    return s, t, res, R


def remove_vertices_update(n: int, src, dst, k: int, R_prev, **kw):
    """The k highest ids removed with every incident edge, ranks of the
    others rescaled, then DF from the marks of those edge deletions: for
    every source u of a removed edge, u itself (self-loop) and its previous
    out-neighbours, among the remaining vertices.  Returns (new_src,
    new_dst, DFResult, rescaled ranks)."""
    n1 = n - k
    src = np.asarray(src, np.int32)
    dst = np.asarray(dst, np.int32)
    e = edge_set(n, src, dst)
    s0, t0 = split_keys(n, e)
    keep = (s0 < n1) & (t0 < n1)
    sources = np.unique(s0[~keep])
    marks = np.zeros(n1, np.uint8)
    out_prev = t0[np.isin(s0, sources)]
    marks[out_prev[out_prev < n1]] = 1
    marks[sources[sources < n1]] = 1
    R = rescale(R_prev, n1)
    s1, t1 = s0[keep], t0[keep]
    res = df_bb(n1, (s1, t1), (s1, t1), np.empty(0, np.int32), R,
                marks=marks, **kw)
    return s1, t1, res, R
