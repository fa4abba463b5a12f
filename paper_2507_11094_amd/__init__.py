"""Python binding of the MI355X dynamic-graph library (include/dg.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels of
libdg.so.  The functions keep the C names (dg_graph_create, dg_apply_batch, ...);
the Graph / Query classes wrap them for convenience.  Arrays are numpy (host
memory) or torch CUDA tensors (device memory, passed with DG_DEVICE_PTRS).

Importing this package fails loudly when libdg.so has not been built: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK = 0
DG_EINVAL = -1
DG_ENOMEM = -2
DG_EDEVICE = -3
DG_ESTATE = -4
DG_EBUSY = -5
DG_EBUDGET = -6
DG_ENOTFOUND = -7
DG_INF = 1073741823
DG_DIRECTED = 0
DG_UNDIRECTED = 1
DG_DEVICE_PTRS = 2

# Every symbol include/dg.h declares (checked by the tests against the .so).
EXPORTS = (
    "dg_last_error", "dg_set_allocator", "dg_graph_create", "dg_graph_destroy",
    "dg_graph_set_stream", "dg_graph_info", "dg_graph_export", "dg_graph_merge",
    "dg_apply_batch", "dg_snapshot_save", "dg_snapshot_restore", "dg_snapshot_free",
    "dg_sssp_attach", "dg_pr_attach", "dg_tc_attach", "dg_query_detach", "dg_sssp_read",
    "dg_pr_read", "dg_tc_read", "dg_sssp_static", "dg_pr_static", "dg_tc_static",
    "dg_profile_enable", "dg_profile_reset", "dg_profile_read",
)


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("merge_threshold", ctypes.c_double), ("pr_tol_scale", ctypes.c_double),
                ("heavy_degree", ctypes.c_int32), ("persistent_groups", ctypes.c_int32),
                ("sssp_persistent", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


class KernelProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class BatchStats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64), ("deleted", ctypes.c_int64),
                ("inserted", ctypes.c_int64), ("ignored_del", ctypes.c_int64),
                ("ignored_ins", ctypes.c_int64), ("diff_entries", ctypes.c_int64),
                ("tombstones", ctypes.c_int64), ("merged", ctypes.c_int32),
                ("chunks", ctypes.c_int32), ("sssp_invalidated", ctypes.c_int64),
                ("sssp_relaxed", ctypes.c_int64), ("sssp_steps", ctypes.c_int32),
                ("pr_iterations", ctypes.c_int32), ("pr_affected", ctypes.c_int64),
                ("edges_traversed", ctypes.c_int64), ("tc_removed", ctypes.c_int64),
                ("tc_added", ctypes.c_int64), ("t_validate_ms", ctypes.c_float),
                ("t_update_ms", ctypes.c_float), ("t_merge_ms", ctypes.c_float),
                ("t_sssp_ms", ctypes.c_float), ("t_pr_ms", ctypes.c_float),
                ("t_tc_ms", ctypes.c_float), ("t_total_ms", ctypes.c_float),
                ("reserved_f", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("reserved")}


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libdg.so (built by paper_2507_11094_amd/build.py).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python paper_2507_11094_amd/build.py)")
    # One HIP runtime per process: load PyTorch's first so libdg.so binds to the
    # libamdhip64.so.7 it already mapped (same SONAME) and device pointers, streams
    # and the device context are shared with torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U32, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    sig = {
        "dg_last_error": ([], ctypes.c_char_p),
        "dg_set_allocator": ([P, P, P], ctypes.c_int),
        "dg_graph_create": ([I32, I64, P, P, P, U32, P, ctypes.POINTER(P)], ctypes.c_int),
        "dg_graph_destroy": ([P], ctypes.c_int),
        "dg_graph_set_stream": ([P, P], ctypes.c_int),
        "dg_graph_info": ([P, P, P, P, P], ctypes.c_int),
        "dg_graph_export": ([P, P, P, P, P], ctypes.c_int),
        "dg_graph_merge": ([P], ctypes.c_int),
        "dg_apply_batch": ([P, I64, P, P, P, P, I64, U32, P], ctypes.c_int),
        "dg_snapshot_save": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "dg_snapshot_restore": ([P, P], ctypes.c_int),
        "dg_snapshot_free": ([P], ctypes.c_int),
        "dg_sssp_attach": ([P, I32, ctypes.POINTER(P)], ctypes.c_int),
        "dg_pr_attach": ([P, D, D, I32, ctypes.POINTER(P)], ctypes.c_int),
        "dg_tc_attach": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "dg_query_detach": ([P], ctypes.c_int),
        "dg_sssp_read": ([P, P, P, U32], ctypes.c_int),
        "dg_pr_read": ([P, P, P, P, U32], ctypes.c_int),
        "dg_tc_read": ([P, P], ctypes.c_int),
        "dg_sssp_static": ([P, I32, P, P, U32], ctypes.c_int),
        "dg_pr_static": ([P, D, D, I32, P, P, U32], ctypes.c_int),
        "dg_tc_static": ([P, P], ctypes.c_int),
        "dg_profile_enable": ([I32], ctypes.c_int),
        "dg_profile_reset": ([], ctypes.c_int),
        "dg_profile_read": ([P, I32, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != DG_OK:
        msg = load_library().dg_last_error()
        raise DGError(rc, msg.decode() if msg else "")


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _arr(a, dtype):
    """(pointer, keepalive, on_device) for a numpy array or a torch tensor."""
    if a is None:
        return None, None, False
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), a, a.is_cuda
    x = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return ctypes.c_void_p(x.ctypes.data), x, False


# ---------------------------------------------------------------------------- C names

def dg_graph_create(n, src, dst, w=None, flags=DG_DIRECTED, cfg: Config | None = None):
    lib = load_library()
    ps, ks, ds = _arr(src, np.int32)
    pd, kd, dd = _arr(dst, np.int32)
    pw, kw, dw = _arr(w, np.int32)
    m = int(ks.numel() if _is_torch(ks) else ks.size)
    if ds:
        flags |= DG_DEVICE_PTRS
    out = ctypes.c_void_p()
    _check(lib.dg_graph_create(int(n), m, ps, pd, pw, flags,
                               ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(out)))
    return out


def dg_apply_batch(g, src, dst, w, op, batch_size=0):
    lib = load_library()
    ps, ks, dev = _arr(src, np.int32)
    pd, kd, _ = _arr(dst, np.int32)
    pw, kw, _ = _arr(w, np.int32)
    po, ko, _ = _arr(op, np.uint8)
    k = int(ks.numel() if _is_torch(ks) else ks.size)
    st = BatchStats()
    _check(lib.dg_apply_batch(g, k, ps, pd, pw, po, int(batch_size),
                              DG_DEVICE_PTRS if dev else 0, ctypes.byref(st)))
    return st


def dg_profile_enable(on: bool = True):
    _check(load_library().dg_profile_enable(1 if on else 0))


def dg_profile_reset():
    _check(load_library().dg_profile_reset())


def dg_profile_read() -> dict:
    """{kernel: {"launches", "ms", "bytes"}} of the launches timed so far."""
    lib = load_library()
    buf = (KernelProf * 64)()
    cnt = ctypes.c_int32()
    _check(lib.dg_profile_read(buf, 64, ctypes.byref(cnt)))
    return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms, "bytes": buf[i].bytes}
            for i in range(min(cnt.value, 64))}


# ---------------------------------------------------------------------------- classes

class Query:
    def __init__(self, graph: "Graph", handle, kind: str):
        self.graph, self.handle, self.kind = graph, handle, kind

    def read(self, out=None, parent=None):
        """SSSP: (dist, parent) int32; PR: (rank, iters, converged); TC: count."""
        lib = load_library()
        n = self.graph.n
        if self.kind == "sssp":
            if out is not None:  # device tensors
                _check(lib.dg_sssp_read(self.handle, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(parent.data_ptr()) if parent is not None else None,
                                        DG_DEVICE_PTRS))
                return out, parent
            dist = np.empty(n, np.int32)
            par = np.empty(n, np.int32)
            _check(lib.dg_sssp_read(self.handle, dist.ctypes.data, par.ctypes.data, 0))
            return dist, par
        if self.kind == "pr":
            it = ctypes.c_int32()
            cv = ctypes.c_int32()
            if out is not None:
                _check(lib.dg_pr_read(self.handle, ctypes.c_void_p(out.data_ptr()), ctypes.byref(it),
                                      ctypes.byref(cv), DG_DEVICE_PTRS))
                return out, it.value, bool(cv.value)
            rank = np.empty(n, np.float64)
            _check(lib.dg_pr_read(self.handle, rank.ctypes.data, ctypes.byref(it), ctypes.byref(cv), 0))
            return rank, it.value, bool(cv.value)
        c = ctypes.c_uint64()
        _check(lib.dg_tc_read(self.handle, ctypes.byref(c)))
        return int(c.value)

    def detach(self):
        if self.handle:
            _check(load_library().dg_query_detach(self.handle))
            self.handle = None


class Graph:
    """A device-resident dynamic graph (diff-CSR, forward + reverse)."""

    def __init__(self, n, src, dst, w=None, undirected=False, config: Config | None = None):
        self.n = int(n)
        self.undirected = bool(undirected)
        self.handle = dg_graph_create(n, src, dst, w, DG_UNDIRECTED if undirected else DG_DIRECTED,
                                      config)
        self._snap = None

    def close(self):
        if getattr(self, "handle", None):
            lib = load_library()
            if self._snap:
                lib.dg_snapshot_free(self._snap)
                self._snap = None
            _check(lib.dg_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_ptr: int):
        _check(load_library().dg_graph_set_stream(self.handle, ctypes.c_void_p(stream_ptr)))

    def apply(self, src, dst, w, op, batch_size=0) -> BatchStats:
        return dg_apply_batch(self.handle, src, dst, w, op, batch_size)

    def info(self):
        n = ctypes.c_int32()
        m = ctypes.c_int64()
        d = ctypes.c_int64()
        t = ctypes.c_int64()
        _check(load_library().dg_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                            ctypes.byref(d), ctypes.byref(t)))
        return {"n": n.value, "m": m.value, "diff_entries": d.value, "tombstones": t.value}

    def export(self):
        lib = load_library()
        m = ctypes.c_int64()
        _check(lib.dg_graph_export(self.handle, ctypes.byref(m), None, None, None))
        s = np.empty(max(m.value, 1), np.int32)
        d = np.empty(max(m.value, 1), np.int32)
        w = np.empty(max(m.value, 1), np.int32)
        _check(lib.dg_graph_export(self.handle, ctypes.byref(m), s.ctypes.data, d.ctypes.data,
                                   w.ctypes.data))
        return s[:m.value].copy(), d[:m.value].copy(), w[:m.value].copy()

    def merge(self):
        _check(load_library().dg_graph_merge(self.handle))

    def snapshot(self):
        lib = load_library()
        if self._snap:
            lib.dg_snapshot_free(self._snap)
        s = ctypes.c_void_p()
        _check(lib.dg_snapshot_save(self.handle, ctypes.byref(s)))
        self._snap = s

    def restore(self):
        _check(load_library().dg_snapshot_restore(self.handle, self._snap))

    def sssp_attach(self, source: int) -> Query:
        q = ctypes.c_void_p()
        _check(load_library().dg_sssp_attach(self.handle, int(source), ctypes.byref(q)))
        return Query(self, q, "sssp")

    def pr_attach(self, damping=0.85, tol=1e-9, max_iter=1000) -> Query:
        q = ctypes.c_void_p()
        _check(load_library().dg_pr_attach(self.handle, float(damping), float(tol), int(max_iter),
                                           ctypes.byref(q)))
        return Query(self, q, "pr")

    def tc_attach(self) -> Query:
        q = ctypes.c_void_p()
        _check(load_library().dg_tc_attach(self.handle, ctypes.byref(q)))
        return Query(self, q, "tc")

    def sssp_static(self, source: int):
        dist = np.empty(self.n, np.int32)
        par = np.empty(self.n, np.int32)
        _check(load_library().dg_sssp_static(self.handle, int(source), dist.ctypes.data,
                                             par.ctypes.data, 0))
        return dist, par

    def pr_static(self, damping=0.85, tol=1e-9, max_iter=1000):
        rank = np.empty(self.n, np.float64)
        it = ctypes.c_int32()
        _check(load_library().dg_pr_static(self.handle, float(damping), float(tol), int(max_iter),
                                           rank.ctypes.data, ctypes.byref(it), 0))
        return rank, it.value

    def tc_static(self) -> int:
        c = ctypes.c_uint64()
        _check(load_library().dg_tc_static(self.handle, ctypes.byref(c)))
        return int(c.value)
