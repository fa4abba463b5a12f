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
DG_INCREMENTAL = 4
DG_DECREMENTAL = 8
DG_NOALLOC_MAX_HOST_N = 522240

# Every symbol include/dg.h declares (checked by the tests against the .so).
EXPORTS = (
    "dg_last_error", "dg_set_allocator", "dg_graph_create", "dg_graph_destroy",
    "dg_graph_set_stream", "dg_graph_info", "dg_graph_export", "dg_graph_merge",
    "dg_apply_batch", "dg_snapshot_save", "dg_snapshot_restore", "dg_snapshot_free",
    "dg_sssp_attach", "dg_pr_attach", "dg_tc_attach", "dg_query_detach", "dg_sssp_read",
    "dg_query_export", "dg_query_import", "dg_pr_read_noalloc", "dg_sort_pairs", "dg_scan_exclusive", "dg_calibrate",
    "dg_pr_gather_floor",
    "dg_pr_read", "dg_tc_read", "dg_sssp_static", "dg_pr_static", "dg_tc_static",
    "dg_profile_enable", "dg_profile_reset", "dg_profile_read",
    "dg_set_create", "dg_set_destroy", "dg_set_info", "dg_set_sssp_attach", "dg_set_apply_sssp",
    "dg_set_sssp_read", "dg_set_graph_stats", "dg_autotune", "dg_set_autotune",
    "dg_server_create", "dg_server_add_graph", "dg_server_start", "dg_server_submit", "dg_server_wait",
    "dg_server_poll", "dg_server_stats", "dg_server_destroy",
)


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("merge_threshold", ctypes.c_double), ("pr_tol_scale", ctypes.c_double),
                ("heavy_degree", ctypes.c_int32), ("persistent_groups", ctypes.c_int32),
                ("sssp_persistent", ctypes.c_int32), ("pr_mode", ctypes.c_int32),
                ("pr_pull", ctypes.c_int32), ("sssp_delta", ctypes.c_int32), ("merge_period", ctypes.c_int32),
                ("pr_tile", ctypes.c_int32), ("merge_tile", ctypes.c_int32), ("vertex_order", ctypes.c_int32),
                ("diff_only", ctypes.c_int32), ("pr_extrapolate", ctypes.c_int32)]


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
                ("pr_moves", ctypes.c_int32)]

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
        "dg_query_export": ([P, P, P], ctypes.c_int),
        "dg_pr_read_noalloc": ([P, P, P, P, U32], ctypes.c_int),
        "dg_sort_pairs": ([P, P, P, P, I64, I32, P], ctypes.c_int),
        "dg_scan_exclusive": ([P, P, I64, P], ctypes.c_int),
        "dg_calibrate": ([I32, P, I64, P], ctypes.c_int),
        "dg_pr_gather_floor": ([P, I32, ctypes.POINTER(D)], ctypes.c_int),
        "dg_query_import": ([P, P, I64, ctypes.POINTER(P)], ctypes.c_int),
        "dg_sssp_static": ([P, I32, P, P, U32], ctypes.c_int),
        "dg_pr_static": ([P, D, D, I32, P, P, U32], ctypes.c_int),
        "dg_tc_static": ([P, P], ctypes.c_int),
        "dg_profile_enable": ([I32], ctypes.c_int),
        "dg_profile_reset": ([], ctypes.c_int),
        "dg_profile_read": ([P, I32, P], ctypes.c_int),
        "dg_set_create": ([I32, P, P, P, P, P, U32, P, ctypes.POINTER(P)], ctypes.c_int),
        "dg_set_destroy": ([P], ctypes.c_int),
        "dg_set_info": ([P, P, P, P], ctypes.c_int),
        "dg_set_sssp_attach": ([P, P], ctypes.c_int),
        "dg_set_apply_sssp": ([P, P, P, P, P, P, U32, P], ctypes.c_int),
        "dg_set_sssp_read": ([P, I32, P, P, U32], ctypes.c_int),
        "dg_set_graph_stats": ([P, P, P], ctypes.c_int),
        "dg_autotune": ([P, I64, P, P, P, P, U32, P, P], ctypes.c_int),
        "dg_set_autotune": ([P, P, P, P, P, P, U32, P, P], ctypes.c_int),
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


def dg_apply_batch(g, src, dst, w, op, batch_size=0, mode=0):
    """mode: 0, DG_INCREMENTAL or DG_DECREMENTAL (op may then be None)."""
    lib = load_library()
    ps, ks, dev = _arr(src, np.int32)
    pd, kd, _ = _arr(dst, np.int32)
    pw, kw, _ = _arr(w, np.int32)
    po, ko, _ = _arr(op, np.uint8)
    k = int(ks.numel() if _is_torch(ks) else ks.size)
    st = BatchStats()
    _check(lib.dg_apply_batch(g, k, ps, pd, pw, po, int(batch_size),
                              (DG_DEVICE_PTRS if dev else 0) | int(mode), ctypes.byref(st)))
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


def dg_sort_pairs(keys, vals, bits=64):
    """Stable radix sort of device tensors (uint64 keys as int64, int32 values) by
    the low `bits` bits of the keys; returns new (keys, values) tensors."""
    import torch

    n = int(keys.numel())
    ko = torch.empty_like(keys)
    vo = torch.empty_like(vals)
    _check(load_library().dg_sort_pairs(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(ko.data_ptr()),
                                        ctypes.c_void_p(vals.data_ptr()), ctypes.c_void_p(vo.data_ptr()), n,
                                        int(bits), None))
    return ko, vo


def dg_scan_exclusive(x):
    """Exclusive prefix sum of an int64 device tensor (new tensor)."""
    import torch

    out = torch.empty_like(x)
    _check(load_library().dg_scan_exclusive(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            int(x.numel()), None))
    return out


# ---------------------------------------------------------------------------- allocator

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_hook = None


class TorchAllocatorHook:
    """dg_set_allocator callbacks that take the library's device memory from
    torch's caching allocator (on the current device and stream).  A free first
    waits for the device, as hipFree does, because the library may free a buffer
    that queued kernels still use.  Counts allocations, frees and live bytes."""

    def __init__(self):
        import torch

        self._torch = torch
        self.allocs = 0
        self.frees = 0
        self._live = {}
        self.c_alloc = _ALLOC_FN(self._alloc)
        self.c_free = _FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None
        self.allocs += 1
        self._live[int(p)] = int(nbytes)
        return p

    def _free(self, p, _ctx):
        if not p:
            return
        self._torch.cuda.synchronize()
        self._torch.cuda.caching_allocator_delete(int(p))
        self.frees += 1
        self._live.pop(int(p), None)

    def live_bytes(self) -> int:
        return sum(self._live.values())


def use_torch_allocator() -> TorchAllocatorHook:
    """Route every device allocation of the library through torch's caching
    allocator (dg_set_allocator; only while no graph, set or server exists)."""
    global _hook
    h = TorchAllocatorHook()
    _check(load_library().dg_set_allocator(ctypes.cast(h.c_alloc, ctypes.c_void_p),
                                           ctypes.cast(h.c_free, ctypes.c_void_p), None))
    _hook = h  # the callbacks must outlive their use
    return h


def use_default_allocator() -> None:
    """Back to hipMalloc / hipFree (only while no graph, set or server exists)."""
    global _hook
    _check(load_library().dg_set_allocator(None, None, None))
    _hook = None


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

    def export(self) -> bytes:
        """The query's state as bytes (dg_query_export), for Graph.import_query."""
        lib = load_library()
        size = ctypes.c_int64()
        _check(lib.dg_query_export(self.handle, None, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        _check(lib.dg_query_export(self.handle, buf, ctypes.byref(size)))
        return buf.raw[:size.value]

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

    def apply(self, src, dst, w, op, batch_size=0, mode=0) -> BatchStats:
        return dg_apply_batch(self.handle, src, dst, w, op, batch_size, mode)

    def insert(self, src, dst, w=None, batch_size=0) -> BatchStats:
        """Incremental-only batch (DG_INCREMENTAL): every update is an insertion."""
        return dg_apply_batch(self.handle, src, dst, w, None, batch_size, DG_INCREMENTAL)

    def delete(self, src, dst, batch_size=0) -> BatchStats:
        """Decremental-only batch (DG_DECREMENTAL): every update is a deletion."""
        return dg_apply_batch(self.handle, src, dst, None, None, batch_size, DG_DECREMENTAL)

    def info(self):
        n = ctypes.c_int32()
        m = ctypes.c_int64()
        d = ctypes.c_int64()
        t = ctypes.c_int64()
        _check(load_library().dg_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                            ctypes.byref(d), ctypes.byref(t)))
        return {"n": n.value, "m": m.value, "diff_entries": d.value, "tombstones": t.value}

    def pr_gather_floor(self, reps: int = 10) -> float:
        """Microseconds per launch of a bare gather over the base reverse columns
        (the floor under the whole-graph PageRank pull)."""
        us = ctypes.c_double()
        _check(load_library().dg_pr_gather_floor(self.handle, int(reps), ctypes.byref(us)))
        return us.value

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

    def import_query(self, blob: bytes) -> Query:
        """Attach a query from Query.export() bytes (dg_query_import)."""
        q = ctypes.c_void_p()
        _check(load_library().dg_query_import(self.handle, blob, len(blob), ctypes.byref(q)))
        kind = {1: "sssp", 2: "pr", 3: "tc"}[int.from_bytes(blob[4:8], "little")]
        return Query(self, q, kind)

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


class GraphSet:
    """Many independent directed graphs updated together (dg_set_*).

    Members are given as lists of (n_i, src_i, dst_i, w_i) with member-local ids."""

    def __init__(self, members, config: Config | None = None):
        lib = load_library()
        self.count = len(members)
        self.n = np.array([m[0] for m in members], np.int32)
        self.m = np.array([len(m[1]) for m in members], np.int64)
        src = np.ascontiguousarray(np.concatenate([np.asarray(m[1], np.int32) for m in members]))
        dst = np.ascontiguousarray(np.concatenate([np.asarray(m[2], np.int32) for m in members]))
        w = np.ascontiguousarray(np.concatenate([np.asarray(m[3], np.int32) for m in members]))
        h = ctypes.c_void_p()
        _check(lib.dg_set_create(self.count, self.n.ctypes.data, self.m.ctypes.data, src.ctypes.data,
                                 dst.ctypes.data, w.ctypes.data, 0,
                                 ctypes.byref(config) if config is not None else None, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(load_library().dg_set_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        c = ctypes.c_int32()
        v = ctypes.c_int64()
        a = ctypes.c_int64()
        _check(load_library().dg_set_info(self.handle, ctypes.byref(c), ctypes.byref(v), ctypes.byref(a)))
        return {"count": c.value, "vertices": v.value, "arcs": a.value}

    def sssp_attach(self, sources):
        s = np.ascontiguousarray(np.asarray(sources, np.int32))
        _check(load_library().dg_set_sssp_attach(self.handle, s.ctypes.data))

    @staticmethod
    def _batches(batches):
        k = np.array([len(b[0]) for b in batches], np.int64)
        cat = [np.ascontiguousarray(np.concatenate([np.asarray(b[i], dt) for b in batches]))
               for i, dt in ((0, np.int32), (1, np.int32), (2, np.int32), (3, np.uint8))]
        return k, cat

    def apply(self, batches) -> BatchStats:
        """batches: per member (src, dst, w, op) with member-local ids."""
        k, (s, d, w, o) = self._batches(batches)
        st = BatchStats()
        _check(load_library().dg_set_apply_sssp(self.handle, k.ctypes.data, s.ctypes.data, d.ctypes.data,
                                                w.ctypes.data, o.ctypes.data, 0, ctypes.byref(st)))
        return st

    def apply_device(self, k, s, d, w, o) -> BatchStats:
        """Pre-concatenated batch already in device memory (torch tensors); k host int64."""
        kk = np.ascontiguousarray(np.asarray(k, np.int64))
        st = BatchStats()
        _check(load_library().dg_set_apply_sssp(self.handle, kk.ctypes.data, ctypes.c_void_p(s.data_ptr()),
                                                ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                                ctypes.c_void_p(o.data_ptr()), DG_DEVICE_PTRS,
                                                ctypes.byref(st)))
        return st

    def autotune(self, batches):
        k, (s, d, w, o) = self._batches(batches)
        best = Config()
        ms = ctypes.c_double()
        _check(load_library().dg_set_autotune(self.handle, k.ctypes.data, s.ctypes.data, d.ctypes.data,
                                              w.ctypes.data, o.ctypes.data, 0, ctypes.byref(best),
                                              ctypes.byref(ms)))
        return best, ms.value

    def read(self, member):
        n = int(self.n[member])
        dist = np.empty(n, np.int32)
        par = np.empty(n, np.int32)
        _check(load_library().dg_set_sssp_read(self.handle, int(member), dist.ctypes.data, par.ctypes.data, 0))
        return dist, par

    def graph_stats(self):
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        _check(load_library().dg_set_graph_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return {"launches": a.value, "captures": b.value}


def autotune(graph: "Graph", src, dst, w, op):
    """dg_autotune on one batch (host arrays); returns (best Config, ms)."""
    ps, ks, _ = _arr(src, np.int32)
    pd, kd, _ = _arr(dst, np.int32)
    pw, kw, _ = _arr(w, np.int32)
    po, ko, _ = _arr(op, np.uint8)
    best = Config()
    ms = ctypes.c_double()
    _check(load_library().dg_autotune(graph.handle, int(ks.size), ps, pd, pw, po, 0, ctypes.byref(best),
                                      ctypes.byref(ms)))
    return best, ms.value


class ServerConfig(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("max_waiting", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int32), ("source", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("k", ctypes.c_int64), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("w", ctypes.c_void_p), ("op", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pr_iters", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("applied", ctypes.c_int64),
                ("tc", ctypes.c_uint64), ("error", ctypes.c_char * 96)]


SSSP, PAGERANK, TRIANGLES = 0, 1, 2


def _server_lib():
    lib = load_library()
    if not getattr(lib, "_server_sigs", False):
        P = ctypes.c_void_p
        for name, args in (("dg_server_create", [P, ctypes.POINTER(P)]),
                           ("dg_server_add_graph", [P, ctypes.c_int32, ctypes.c_int64, P, P, P, P, P]),
                           ("dg_server_start", [P]), ("dg_server_submit", [P, P, P]),
                           ("dg_server_wait", [P, ctypes.c_int64, ctypes.c_double, P]),
                           ("dg_server_poll", [P, ctypes.c_int64, P]), ("dg_server_stats", [P, P, P]),
                           ("dg_server_destroy", [P])):
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib._server_sigs = True
    return lib


class Server:
    """dg_server_*: resident graphs, continuous batching across graphs, admission by
    a device-memory budget."""

    def __init__(self, workers=4, budget_bytes=8 << 30, max_waiting=1 << 20):
        lib = _server_lib()
        c = ServerConfig(workers, 0, budget_bytes, max_waiting)
        h = ctypes.c_void_p()
        _check(lib.dg_server_create(ctypes.byref(c), ctypes.byref(h)))
        self.handle = h
        self.n = []
        self._pending = {}

    def add_graph(self, n, src, dst, w=None, config: Config | None = None) -> int:
        s = np.ascontiguousarray(np.asarray(src, np.int32))
        d = np.ascontiguousarray(np.asarray(dst, np.int32))
        ww = None if w is None else np.ascontiguousarray(np.asarray(w, np.int32))
        gid = ctypes.c_int32()
        _check(_server_lib().dg_server_add_graph(self.handle, int(n), s.size, s.ctypes.data, d.ctypes.data,
                                                 None if ww is None else ww.ctypes.data,
                                                 ctypes.byref(config) if config is not None else None,
                                                 ctypes.byref(gid)))
        self.n.append(int(n))
        return gid.value

    def start(self):
        _check(_server_lib().dg_server_start(self.handle))

    def submit(self, graph, kind, src, dst, w, op, source=0) -> int:
        n = self.n[graph]
        out = (np.empty(n, np.int32) if kind == SSSP else np.empty(n, np.float64) if kind == PAGERANK
               else np.zeros(1, np.uint64))
        arrs = [np.ascontiguousarray(np.asarray(a, dt)) for a, dt in
                ((src, np.int32), (dst, np.int32), (w, np.int32), (op, np.uint8))]
        r = Request(int(graph), int(kind), int(source), 0, arrs[0].size, arrs[0].ctypes.data, arrs[1].ctypes.data,
                    arrs[2].ctypes.data, arrs[3].ctypes.data, out.ctypes.data)
        t = ctypes.c_int64()
        _check(_server_lib().dg_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._pending[t.value] = out  # keep the result buffer alive
        return t.value

    def wait(self, ticket, timeout=-1.0):
        res = Result()
        _check(_server_lib().dg_server_wait(self.handle, int(ticket), float(timeout), ctypes.byref(res)))
        out = self._pending.pop(ticket)
        return res, out

    def stats(self):
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        _check(_server_lib().dg_server_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return {"waiting": a.value, "inflight_bytes": b.value}

    def close(self):
        if getattr(self, "handle", None):
            _check(_server_lib().dg_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
