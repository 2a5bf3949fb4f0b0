"""ctypes binding of libdfpr (include/dfpr.h): argument marshalling only.

Every function of the C ABI has a Python function of the same name.  Arrays
may be numpy arrays (host memory) or torch tensors on the HIP device (device
memory, passed by data pointer); the library's stream is the current torch
stream when torch sees a device.  Negative status codes raise DfprError.

The shared library must have been built (``paper_2407_19562_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DFPR_LIB") or os.path.join(HERE, "libdfpr.so")

DFPR_OK = 0
DFPR_NOTCONVERGED = 1
DFPR_EINVAL = -1
DFPR_ENOMEM = -2
DFPR_EHIP = -3
DFPR_EABORT = -4
DFPR_ESTATE = -5
DFPR_MEM_HOST = 0
DFPR_MEM_DEVICE = 1
DFPR_ASYNC = 0
DFPR_SYNC = 1
DFPR_STOP_TOL = 0
DFPR_STOP_FRONTIER = 1
DFPR_OUT = 0
DFPR_IN = 1

# the symbols include/dfpr.h declares
EXPORTS = (
    "dfpr_params_default", "dfpr_graph_create", "dfpr_graph_destroy",
    "dfpr_set_params", "dfpr_get_params", "dfpr_graph_size", "dfpr_static",
    "dfpr_naive_dynamic", "dfpr_static_lock_free", "dfpr_naive_dynamic_lock_free",
    "dfpr_set_faults",
    "dfpr_set_ranks", "dfpr_read_ranks",
    "dfpr_apply_batch", "dfpr_update", "dfpr_add_vertices",
    "dfpr_remove_vertices", "dfpr_mark_reachable",
    "dfpr_update_traversal", "dfpr_update_many", "dfpr_update_many_noalloc",
    "dfpr_read_edges",
    "dfpr_read_marks", "dfpr_graph_bytes", "dfpr_stream_copy",
    "dfpr_last_kernel_bytes", "dfpr_strerror", "dfpr_last_error",
)


class dfpr_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tol", ctypes.c_double),
                ("frontier_tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("kahan_min_degree", ctypes.c_int32),
                ("split_min_degree", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("renormalize", ctypes.c_int32), ("timeout_ms", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("graph_replay", ctypes.c_int32),
                ("lf_stop", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dfpr_stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("initial_marked", ctypes.c_int64),
                ("affected", ctypes.c_int64),
                ("vertices_processed", ctypes.c_int64),
                ("edges_gathered", ctypes.c_int64),
                ("out_edges_scanned", ctypes.c_int64),
                ("max_delta", ctypes.c_double), ("ms", ctypes.c_float),
                ("ms_kernel", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DfprError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib().dfpr_last_error().decode()
        super().__init__(f"{where}: {_lib().dfpr_strerror(status).decode()}"
                         f" ({status}): {msg}")


_handle = None


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2407_19562_amd.build` (no fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        P, V = ctypes.POINTER, ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        sig = {
            "dfpr_params_default": [P(dfpr_params)],
            "dfpr_graph_create": [i32, i64, V, V, ctypes.c_int,
                                  P(dfpr_params), V, P(V)],
            "dfpr_graph_destroy": [V],
            "dfpr_set_params": [V, P(dfpr_params)],
            "dfpr_get_params": [V, P(dfpr_params)],
            "dfpr_graph_size": [V, P(i32), P(i64)],
            "dfpr_static": [V, P(dfpr_stats)],
            "dfpr_naive_dynamic": [V, P(dfpr_stats)],
            "dfpr_static_lock_free": [V, P(dfpr_stats)],
            "dfpr_naive_dynamic_lock_free": [V, P(dfpr_stats)],
            "dfpr_set_faults": [V, P(ctypes.c_int32), ctypes.c_int32],
            "dfpr_set_ranks": [V, V, ctypes.c_int],
            "dfpr_read_ranks": [V, V, ctypes.c_int],
            "dfpr_apply_batch": [V, i64, V, V, i64, V, V, ctypes.c_int,
                                 P(i64), P(i64)],
            "dfpr_update": [V, P(dfpr_stats)],
            "dfpr_mark_reachable": [V, P(i64)],
            "dfpr_add_vertices": [V, i32, P(i32)],
            "dfpr_remove_vertices": [V, i32],
            "dfpr_update_traversal": [V, P(dfpr_stats)],
            "dfpr_update_many": [V, i32, V],
            "dfpr_update_many_noalloc": [V, i32, V],
            "dfpr_read_edges": [V, ctypes.c_int, V, V, i64, P(i64)],
            "dfpr_read_marks": [V, V, P(i64)],
            "dfpr_graph_bytes": [V, P(i64)],
            "dfpr_stream_copy": [V, V, i64, V, P(ctypes.c_float)],
            "dfpr_last_kernel_bytes": [V, P(ctypes.c_double), P(i32)],
            "dfpr_strerror": [ctypes.c_int],
            "dfpr_last_error": [],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.dfpr_strerror.restype = ctypes.c_char_p
        lib.dfpr_last_error.restype = ctypes.c_char_p
        _handle = lib
    return _handle


def _check(status: int, where: str) -> int:
    if status < 0:
        raise DfprError(status, where)
    return status


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _arr(a, dtype):
    """(pointer, mem, keepalive) for a numpy array or a device tensor."""
    if a is None:
        return None, DFPR_MEM_HOST, None
    if _is_torch(a):
        if not a.is_cuda:
            a = a.numpy()
        else:
            if not a.is_contiguous():
                raise ValueError("device tensors must be contiguous")
            want = {np.int32: "torch.int32", np.float64: "torch.float64"}[dtype]
            if str(a.dtype) != want:
                raise TypeError(f"expected {want}, got {a.dtype}")
            return ctypes.c_void_p(a.data_ptr()), DFPR_MEM_DEVICE, a
    a = np.ascontiguousarray(a, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), DFPR_MEM_HOST, a


def current_stream():
    """The current torch HIP stream handle (None without a device)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


# --- one Python function per C entry point ------------------------------------

def dfpr_params_default(**overrides) -> dfpr_params:
    p = dfpr_params()
    _check(_lib().dfpr_params_default(ctypes.byref(p)), "dfpr_params_default")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def dfpr_graph_create(n: int, src, dst, params: dfpr_params | None = None,
                      stream=None) -> ctypes.c_void_p:
    ps, ms, k1 = _arr(src, np.int32)
    pd, md, k2 = _arr(dst, np.int32)
    m = 0 if src is None else int(src.numel() if _is_torch(src) else np.size(src))
    if ms != md:
        raise ValueError("src and dst must live in the same memory")
    out = ctypes.c_void_p()
    _check(_lib().dfpr_graph_create(
        int(n), m, ps, pd, ms, ctypes.byref(params) if params else None,
        stream if stream is not None else current_stream(), ctypes.byref(out)),
        "dfpr_graph_create")
    return out


def dfpr_graph_destroy(g) -> None:
    _check(_lib().dfpr_graph_destroy(g), "dfpr_graph_destroy")


def dfpr_set_params(g, p: dfpr_params) -> None:
    _check(_lib().dfpr_set_params(g, ctypes.byref(p)), "dfpr_set_params")


def dfpr_get_params(g) -> dfpr_params:
    p = dfpr_params()
    _check(_lib().dfpr_get_params(g, ctypes.byref(p)), "dfpr_get_params")
    return p


def dfpr_graph_size(g):
    n, m = ctypes.c_int32(), ctypes.c_int64()
    _check(_lib().dfpr_graph_size(g, ctypes.byref(n), ctypes.byref(m)),
           "dfpr_graph_size")
    return n.value, m.value


def _stats_call(fn, g, where):
    st = dfpr_stats()
    rc = _check(fn(g, ctypes.byref(st)), where)
    return rc, st


def dfpr_static(g):
    return _stats_call(_lib().dfpr_static, g, "dfpr_static")


def dfpr_naive_dynamic(g):
    return _stats_call(_lib().dfpr_naive_dynamic, g, "dfpr_naive_dynamic")


def dfpr_static_lock_free(g):
    return _stats_call(_lib().dfpr_static_lock_free, g, "dfpr_static_lock_free")


def dfpr_naive_dynamic_lock_free(g):
    return _stats_call(_lib().dfpr_naive_dynamic_lock_free, g,
                       "dfpr_naive_dynamic_lock_free")


def dfpr_set_faults(g, table) -> None:
    """Per-workgroup fault table (see the header): 0 none, > 0 delay in
    microseconds after each claim, -1 stop at a claim boundary."""
    t = np.ascontiguousarray(np.asarray(table if table is not None else [], np.int32))
    _check(_lib().dfpr_set_faults(g, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  int(t.size)), "dfpr_set_faults")


def dfpr_update(g):
    return _stats_call(_lib().dfpr_update, g, "dfpr_update")


def dfpr_add_vertices(g, count: int) -> int:
    first = ctypes.c_int32()
    _check(_lib().dfpr_add_vertices(g, int(count), ctypes.byref(first)),
           "dfpr_add_vertices")
    return int(first.value)


def dfpr_remove_vertices(g, count: int) -> None:
    _check(_lib().dfpr_remove_vertices(g, int(count)), "dfpr_remove_vertices")


def dfpr_mark_reachable(g) -> int:
    c = ctypes.c_int64()
    _check(_lib().dfpr_mark_reachable(g, ctypes.byref(c)), "dfpr_mark_reachable")
    return int(c.value)


def dfpr_update_traversal(g):
    return _stats_call(_lib().dfpr_update_traversal, g, "dfpr_update_traversal")


def dfpr_update_many(graphs):
    arr = (ctypes.c_void_p * len(graphs))(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in graphs])
    stats = (dfpr_stats * len(graphs))()
    rc = _check(_lib().dfpr_update_many(arr, len(graphs), stats),
                "dfpr_update_many")
    return rc, list(stats)


def dfpr_update_many_noalloc(graphs):
    """dfpr_update_many without any allocation (fixed device workspace)."""
    arr = (ctypes.c_void_p * len(graphs))(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in graphs])
    stats = (dfpr_stats * len(graphs))()
    rc = _check(_lib().dfpr_update_many_noalloc(arr, len(graphs), stats),
                "dfpr_update_many_noalloc")
    return rc, list(stats)


DFPR_NOALLOC_MAX_GRAPHS = 4096


def dfpr_set_ranks(g, r) -> None:
    p, mem, keep = _arr(r, np.float64)
    _check(_lib().dfpr_set_ranks(g, p, mem), "dfpr_set_ranks")


def dfpr_read_ranks(g, out=None):
    """Returns the ranks as a float64 numpy array, or fills a device tensor."""
    if out is None:
        n, _ = dfpr_graph_size(g)
        out = np.empty(n, np.float64)
    p, mem, keep = _arr(out, np.float64)
    _check(_lib().dfpr_read_ranks(g, p, mem), "dfpr_read_ranks")
    return out


def dfpr_apply_batch(g, del_src, del_dst, ins_src, ins_dst):
    """Returns (applied_del, applied_ins)."""
    arrs = [_arr(a, np.int32) for a in (del_src, del_dst, ins_src, ins_dst)]
    mems = {mem for (p, mem, k), a in zip(arrs, (del_src, del_dst, ins_src, ins_dst))
            if a is not None and _size(a) > 0}
    if len(mems) > 1:
        raise ValueError("all batch arrays must live in the same memory")
    mem = mems.pop() if mems else DFPR_MEM_HOST
    nd = _size(del_src)
    ni = _size(ins_src)
    if _size(del_dst) != nd or _size(ins_dst) != ni:
        raise ValueError("src/dst lengths differ")
    ad, ai = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib().dfpr_apply_batch(g, nd, arrs[0][0], arrs[1][0], ni,
                                   arrs[2][0], arrs[3][0], mem,
                                   ctypes.byref(ad), ctypes.byref(ai)),
           "dfpr_apply_batch")
    return ad.value, ai.value


def _size(a) -> int:
    if a is None:
        return 0
    return int(a.numel()) if _is_torch(a) else int(np.size(a))


def dfpr_read_edges(g, direction: int = DFPR_OUT):
    cnt = ctypes.c_int64()
    _check(_lib().dfpr_read_edges(g, direction, None, None, 0,
                                  ctypes.byref(cnt)), "dfpr_read_edges")
    s = np.empty(cnt.value, np.int32)
    d = np.empty(cnt.value, np.int32)
    _check(_lib().dfpr_read_edges(g, direction,
                                  s.ctypes.data_as(ctypes.c_void_p),
                                  d.ctypes.data_as(ctypes.c_void_p),
                                  cnt.value, ctypes.byref(cnt)),
           "dfpr_read_edges")
    return s, d


def dfpr_read_marks(g):
    n, _ = dfpr_graph_size(g)
    a = np.empty(n, np.uint8)
    c = ctypes.c_int64()
    _check(_lib().dfpr_read_marks(g, a.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(c)), "dfpr_read_marks")
    return a.astype(bool), c.value


def dfpr_graph_bytes(g) -> int:
    b = ctypes.c_int64()
    _check(_lib().dfpr_graph_bytes(g, ctypes.byref(b)), "dfpr_graph_bytes")
    return b.value


def dfpr_stream_copy(dst, src, nbytes: int, stream=None) -> float:
    ms = ctypes.c_float()
    _check(_lib().dfpr_stream_copy(ctypes.c_void_p(dst.data_ptr()),
                                   ctypes.c_void_p(src.data_ptr()), int(nbytes),
                                   stream if stream is not None else current_stream(),
                                   ctypes.byref(ms)), "dfpr_stream_copy")
    return ms.value


def dfpr_last_kernel_bytes(g):
    b, l = ctypes.c_double(), ctypes.c_int32()
    _check(_lib().dfpr_last_kernel_bytes(g, ctypes.byref(b), ctypes.byref(l)),
           "dfpr_last_kernel_bytes")
    return b.value, l.value


def dfpr_strerror(status: int) -> str:
    return _lib().dfpr_strerror(status).decode()


def dfpr_last_error() -> str:
    return _lib().dfpr_last_error().decode()


# --- convenience wrapper ----------------------------------------------------------

class Graph:
    """Owns one dfpr_graph handle."""

    def __init__(self, n, src, dst, params: dfpr_params | None = None,
                 stream=None, **overrides):
        if params is None:
            params = dfpr_params_default(**overrides)
        self.params = params
        self.h = dfpr_graph_create(n, src, dst, params, stream)
        self.n = int(n)

    def close(self):
        if self.h:
            dfpr_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, **kw):
        p = dfpr_get_params(self.h)
        for k, v in kw.items():
            setattr(p, k, v)
        dfpr_set_params(self.h, p)
        self.params = p

    def static(self):
        return dfpr_static(self.h)

    def naive_dynamic(self):
        return dfpr_naive_dynamic(self.h)

    def static_lock_free(self):
        return dfpr_static_lock_free(self.h)

    def naive_dynamic_lock_free(self):
        return dfpr_naive_dynamic_lock_free(self.h)

    def set_faults(self, table):
        dfpr_set_faults(self.h, table)

    def apply_batch(self, del_src, del_dst, ins_src, ins_dst):
        return dfpr_apply_batch(self.h, del_src, del_dst, ins_src, ins_dst)

    def apply(self, batch):
        return self.apply_batch(batch.del_src, batch.del_dst, batch.ins_src,
                                batch.ins_dst)

    def update(self):
        return dfpr_update(self.h)

    def add_vertices(self, count: int) -> int:
        """Appends `count` isolated vertices; returns the first new id."""
        first = dfpr_add_vertices(self.h, count)
        self.n, _ = dfpr_graph_size(self.h)
        return first

    def remove_vertices(self, count: int) -> None:
        """Removes the `count` highest ids with their edges."""
        dfpr_remove_vertices(self.h, count)
        self.n, _ = dfpr_graph_size(self.h)

    def mark_reachable(self) -> int:
        return dfpr_mark_reachable(self.h)

    def update_traversal(self):
        return dfpr_update_traversal(self.h)

    def ranks(self, out=None):
        return dfpr_read_ranks(self.h, out)

    def set_ranks(self, r):
        dfpr_set_ranks(self.h, r)

    def edges(self, direction=DFPR_OUT):
        return dfpr_read_edges(self.h, direction)

    def marks(self):
        return dfpr_read_marks(self.h)

    def size(self):
        return dfpr_graph_size(self.h)

    def kernel_bytes(self):
        return dfpr_last_kernel_bytes(self.h)
