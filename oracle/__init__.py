"""CPU oracle: apply an update batch to an edge set, then recompute statically.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
links or calls it, and it imports nothing from the GPU library.

The arithmetic lives in ``oracle.c`` (plain single-threaded C, fp64 for PageRank,
64-bit sums for shortest paths, uint64 triangle counts); this module only
compiles it with gcc and marshals numpy arrays.  Function comments in the C file
cite the paper passages they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

INF = 1073741823  # unreachable distance, INT_MAX / 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with plain gcc -O2 (no OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _i32p():
    return np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    i32p = _i32p()
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.orc_apply.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p,
                              ctypes.c_int64, i32p, i32p, i32p, u8p, i32p, i32p, i32p,
                              ctypes.c_int64, i64p]
    lib.orc_apply.restype = ctypes.c_int64
    lib.orc_sssp.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, ctypes.c_int32, i32p]
    lib.orc_sssp.restype = ctypes.c_int
    lib.orc_pagerank.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int32, f64p,
                                 ctypes.POINTER(ctypes.c_int32)]
    lib.orc_pagerank.restype = ctypes.c_int
    lib.orc_tc.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p,
                           ctypes.POINTER(ctypes.c_uint64)]
    lib.orc_tc.restype = ctypes.c_int
    lib.orc_symmetrise.argtypes = [ctypes.c_int64, i32p, i32p, i32p, i32p]
    lib.orc_symmetrise.restype = ctypes.c_int64
    _lib = lib
    return lib


def _c32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class InvalidBatch(ValueError):
    """The batch holds a self-loop, an out-of-range id, a bad op or weight."""


def apply(n, src, dst, w, bsrc, bdst, bw, bop, undirected=False):
    """G' = (E \\ D) U A.  Returns (src', dst', w', stats) sorted by (src, dst);
    stats = (applied deletions, applied insertions, ignored deletions, ignored
    insertions).  Undirected edges come back once each as (min, max)."""
    src, dst = _c32(src), _c32(dst)
    w = _c32(np.ones(src.size, np.int32) if w is None else w)
    bsrc, bdst, bw = _c32(bsrc), _c32(bdst), _c32(bw)
    bop = np.ascontiguousarray(np.asarray(bop, dtype=np.uint8))
    cap = src.size + bsrc.size + 1
    os_, od, ow = (np.empty(cap, np.int32) for _ in range(3))
    stats = np.zeros(4, np.int64)
    r = _load().orc_apply(int(n), int(bool(undirected)), src.size, src, dst, w, bsrc.size,
                          bsrc, bdst, bw, bop, os_, od, ow, cap, stats)
    if r == -1:
        raise InvalidBatch("batch rejected")
    if r < 0:
        raise ValueError(f"orc_apply failed ({r})")
    return os_[:r].copy(), od[:r].copy(), ow[:r].copy(), tuple(int(x) for x in stats)


def sssp(n, src, dst, w, source):
    """Shortest distances from ``source`` (int32, INF when unreachable)."""
    src, dst, w = _c32(src), _c32(dst), _c32(w)
    dist = np.empty(int(n), np.int32)
    r = _load().orc_sssp(int(n), src.size, src, dst, w, int(source), dist)
    if r != 0:
        raise ValueError(f"orc_sssp failed ({r})")
    return dist


def pagerank(n, src, dst, damping=0.85, tol=1e-9, max_iter=1000):
    """Normalised FP64 PageRank; returns (rank, iterations, converged)."""
    src, dst = _c32(src), _c32(dst)
    rank = np.empty(int(n), np.float64)
    it = ctypes.c_int32(0)
    r = _load().orc_pagerank(int(n), src.size, src, dst, float(damping), float(tol),
                             int(max_iter), rank, ctypes.byref(it))
    if r < 0:
        raise ValueError("orc_pagerank failed")
    return rank, int(it.value), r == 0


def triangles(n, u, v) -> int:
    """Exact triangle count of the undirected graph with edges {u[i], v[i]}."""
    u, v = _c32(u), _c32(v)
    c = ctypes.c_uint64(0)
    if _load().orc_tc(int(n), u.size, u, v, ctypes.byref(c)) != 0:
        raise ValueError("orc_tc failed")
    return int(c.value)


def symmetrise(src, dst):
    """Undirected view of a directed edge set: each {u, v} once as (min, max)."""
    src, dst = _c32(src), _c32(dst)
    ou = np.empty(max(src.size, 1), np.int32)
    ov = np.empty(max(src.size, 1), np.int32)
    c = _load().orc_symmetrise(src.size, src, dst, ou, ov)
    return ou[:c].copy(), ov[:c].copy()
