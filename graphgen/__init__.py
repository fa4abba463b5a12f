"""Seeded synthetic inputs for the dynamic-graph workloads.

This module is shared by the CPU oracle, the GPU tests and the benchmark.  It
holds no arithmetic of the method itself (no shortest paths, ranks or triangle
counts): it only draws graphs and update batches.

Random numbers come from a counter-based SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): value ``i`` of a
stream is the SplitMix64 finaliser applied to ``seed + (i + 1) * golden``, so any
sub-range of a stream can be drawn independently and every draw is reproducible.

Workload shapes follow the paper's evaluation (Section 6, graph inputs table):
R-MAT graphs with a = 0.57, b = 0.19, c = 0.19, d = 0.05, a 4-neighbour grid as
the road-network stand-in, and update batches expressed as a percentage of |E|
with inserts and deletes counted together.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Distinct sub-stream tags so that every quantity of a workload has its own stream.
_TAG = {
    "rmat": 0x52, "w": 0x57, "del": 0x44, "ins_u": 0x49, "ins_v": 0x4A,
    "ins_w": 0x4B, "perm": 0x50, "orient": 0x4F, "misc": 0x4D,
    # workload-level draws: member scales and batch fractions of a graph set,
    # request arrival gaps, target graph, batch size, query kind and source
    "scale": 0x53, "frac": 0x46, "gap": 0x47, "graph": 0x67, "k": 0x6B, "kind": 0x71,
    "source": 0x73,
}

BASE_SEED = 0xD15C0


def config_seed(config_index: int, instance: int = 0) -> int:
    """Seed of one workload instance: ``0xD15C0 + 1000 * config_index + instance``."""
    return BASE_SEED + 1000 * int(config_index) + int(instance)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_seed(seed: int, tag: str | int) -> int:
    """Derive the seed of a named sub-stream (one SplitMix64 step on seed ^ tag)."""
    t = _TAG[tag] if isinstance(tag, str) else int(tag)
    with np.errstate(over="ignore"):
        z = np.array([((int(seed) * 0x100000001B3) ^ (t << 48) ^ t) & _MASK64], dtype=np.uint64)
        return int(_mix(z + GOLDEN)[0])


def draws(seed: int, start: int, count: int) -> np.ndarray:
    """``count`` uint64 values of the stream ``seed`` starting at counter ``start``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        return _mix(np.uint64(seed & _MASK64) + i * GOLDEN)


def uniform_int(seed: int, start: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi] (inclusive); modulo bias is below 2^-40 here."""
    span = np.uint64(hi - lo + 1)
    return (draws(seed, start, count) % span).astype(np.int64) + lo


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    return (draws(seed, start, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


# ----------------------------------------------------------------------------- R-MAT

def _rmat_candidates(seed: int, scale: int, start: int, count: int, a: float, b: float, c: float):
    """R-MAT endpoint pairs for candidates ``start .. start+count``.

    Each level takes a 16-bit slice of a draw and picks a quadrant with
    probabilities (a, b, c, d); vertex ids are built most-significant bit first
    and are not permuted, so vertex 0 is the densest hub.
    """
    words = (scale + 3) // 4
    ta = np.uint64(int(round(a * 65536)))
    tab = np.uint64(int(round((a + b) * 65536)))
    tabc = np.uint64(int(round((a + b + c) * 65536)))
    src = np.zeros(count, dtype=np.int64)
    dst = np.zeros(count, dtype=np.int64)
    s = stream_seed(seed, "rmat")
    level = 0
    for j in range(words):
        # word j of candidate i is counter i * words + j
        with np.errstate(over="ignore"):
            idx = (np.arange(start, start + count, dtype=np.uint64) * np.uint64(words) + np.uint64(j + 1))
            wv = _mix(np.uint64(s) + idx * GOLDEN)
        for q in range(4):
            if level >= scale:
                break
            r = (wv >> np.uint64(16 * q)) & np.uint64(0xFFFF)
            sbit = (r >= tab).astype(np.int64)              # quadrants c, d
            dbit = ((r >= ta) & (r < tab)) | (r >= tabc)     # quadrants b, d
            src = (src << 1) | sbit
            dst = (dst << 1) | dbit.astype(np.int64)
            level += 1
    return src, dst


def _first_unique(keys: np.ndarray, want: int) -> np.ndarray:
    """Positions of the first occurrence of each distinct key, in draw order,
    truncated to ``want`` entries."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return first[:want]


# The C core computes exactly the numpy definitions above, only faster; the
# numpy versions stay as the definition the tests compare it against.
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile the C core of the generator (plain gcc, OpenMP)."""
    src = os.path.join(_HERE, "rmat.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _native():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_native())
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        lib.gg_rmat_candidates.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32, i64p, i64p]
        lib.gg_rmat_candidates.restype = None
        lib.gg_first_unique.argtypes = [u64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, i64p]
        lib.gg_first_unique.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _rmat_candidates_fast(seed, scale, start, count, a, b, c):
    s = np.empty(count, np.int64)
    d = np.empty(count, np.int64)
    _native().gg_rmat_candidates(stream_seed(seed, "rmat"), scale, start, count,
                                 int(round(a * 65536)), int(round((a + b) * 65536)),
                                 int(round((a + b + c) * 65536)), s, d)
    return s, d


def _first_unique_fast(keys: np.ndarray, want: int, key_bits: int) -> np.ndarray:
    out = np.empty(min(want, keys.size), np.int64)
    k = np.ascontiguousarray(keys.astype(np.uint64))
    c = _native().gg_first_unique(k, k.size, int(key_bits), int(want), out)
    return out[:c]


def rmat_directed(scale: int, m: int, seed: int, wmax: int = 100,
                  a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """Directed simple R-MAT graph with exactly ``m`` distinct arcs, no self-loops,
    int32 weights uniform in [1, wmax].  Returns (n, src, dst, w) as int32 arrays in
    draw order."""
    n = 1 << scale
    if m > n * (n - 1):
        raise ValueError("too many arcs for a simple graph")
    got_s = np.empty(0, np.int64)
    got_d = np.empty(0, np.int64)
    start = 0
    batch = int(m * 1.25) + 1024
    while True:
        s, d = _rmat_candidates_fast(seed, scale, start, batch, a, b, c)
        start += batch
        keep = s != d
        got_s = np.concatenate([got_s, s[keep]])
        got_d = np.concatenate([got_d, d[keep]])
        keys = (got_s << scale) | got_d
        first = _first_unique_fast(keys, m, 2 * scale)
        if first.size >= m:
            got_s, got_d = got_s[first], got_d[first]
            break
        got_s, got_d = got_s[first], got_d[first]
        batch = max(1024, int((m - first.size) * 2.0))
    w = uniform_int(stream_seed(seed, "w"), 0, m, 1, wmax)
    return n, got_s.astype(np.int32), got_d.astype(np.int32), w.astype(np.int32)


def rmat_undirected(scale: int, m_undirected: int, seed: int,
                    a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """Undirected simple R-MAT graph with exactly ``m_undirected`` distinct edges,
    each returned once as a pair (u, v) with u < v.  Returns (n, u, v)."""
    n = 1 << scale
    got_u = np.empty(0, np.int64)
    got_v = np.empty(0, np.int64)
    start = 0
    batch = int(m_undirected * 1.4) + 1024
    while True:
        s, d = _rmat_candidates_fast(seed, scale, start, batch, a, b, c)
        start += batch
        keep = s != d
        u = np.minimum(s[keep], d[keep])
        v = np.maximum(s[keep], d[keep])
        got_u = np.concatenate([got_u, u])
        got_v = np.concatenate([got_v, v])
        first = _first_unique_fast((got_u << scale) | got_v, m_undirected, 2 * scale)
        got_u, got_v = got_u[first], got_v[first]
        if first.size >= m_undirected:
            break
        batch = max(1024, int((m_undirected - first.size) * 3.0))
    return n, got_u.astype(np.int32), got_v.astype(np.int32)


# ----------------------------------------------------------------------------- grid

def grid4(rows: int, cols: int, seed: int, wmax: int = 1000):
    """4-neighbour grid (road-network stand-in).  Vertex (r, c) has id r*cols + c.
    Each undirected edge gets one weight uniform in [1, wmax], shared by both arcs.
    Returns (n, src, dst, w) with both arcs of every edge."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64).reshape(rows, cols)
    hu = ids[:, :-1].ravel(); hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel(); vv = ids[1:, :].ravel()
    u = np.concatenate([hu, vu]); v = np.concatenate([hv, vv])
    w = uniform_int(stream_seed(seed, "w"), 0, u.size, 1, wmax)
    src = np.concatenate([u, v]).astype(np.int32)
    dst = np.concatenate([v, u]).astype(np.int32)
    ww = np.concatenate([w, w]).astype(np.int32)
    return n, src, dst, ww


# ----------------------------------------------------------------------------- batches

def _sorted_keys(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    k = (src.astype(np.int64) << 32) | dst.astype(np.int64)
    k.sort()
    return k


def _contains(sorted_keys: np.ndarray, keys: np.ndarray) -> np.ndarray:
    if sorted_keys.size == 0:
        return np.zeros(keys.shape, dtype=bool)
    pos = np.searchsorted(sorted_keys, keys)
    pos = np.minimum(pos, sorted_keys.size - 1)
    return sorted_keys[pos] == keys


def _distinct_indices(seed: int, m: int, want: int) -> np.ndarray:
    """``want`` distinct indices uniform in [0, m), in draw order."""
    if want > m:
        raise ValueError("cannot delete more edges than exist")
    got = np.empty(0, np.int64)
    start = 0
    while got.size < want:
        need = want - got.size
        cand = uniform_int(seed, start, int(need * 1.2) + 64, 0, m - 1)
        start += cand.size
        got = np.concatenate([got, cand])
        got = got[_first_unique(got, want)]
    return got


def _new_pairs(seed: int, n: int, want: int, existing_sorted: np.ndarray, undirected: bool):
    """``want`` uniform random vertex pairs (u != v) absent from the graph and
    distinct among themselves, in draw order."""
    cap = n * (n - 1) // (2 if undirected else 1)
    if want > cap - existing_sorted.size:
        raise ValueError("not enough absent vertex pairs for the requested insertions")
    su, sv = stream_seed(seed, "ins_u"), stream_seed(seed, "ins_v")
    got_u = np.empty(0, np.int64)
    got_v = np.empty(0, np.int64)
    start = 0
    while got_u.size < want:
        cnt = int((want - got_u.size) * 1.3) + 64
        u = uniform_int(su, start, cnt, 0, n - 1)
        v = uniform_int(sv, start, cnt, 0, n - 1)
        start += cnt
        keep = u != v
        u, v = u[keep], v[keep]
        if undirected:
            u, v = np.minimum(u, v), np.maximum(u, v)
        keys = (u << 32) | v
        fresh = ~_contains(existing_sorted, keys)
        got_u = np.concatenate([got_u, u[fresh]])
        got_v = np.concatenate([got_v, v[fresh]])
        first = _first_unique((got_u << 32) | got_v, want)
        got_u, got_v = got_u[first], got_v[first]
    return got_u, got_v


def edge_keys(src: np.ndarray, dst: np.ndarray, undirected: bool = False) -> np.ndarray:
    """Sorted int64 keys (u << 32 | v) of an edge list (u < v when undirected);
    pass to update_batch to avoid re-sorting a large graph for every batch."""
    if undirected:
        return _sorted_keys(np.minimum(src, dst).astype(np.int64), np.maximum(src, dst).astype(np.int64))
    return _sorted_keys(src, dst)


def update_batch(n: int, src: np.ndarray, dst: np.ndarray, k: int, seed: int,
                 wmax: int = 100, undirected: bool = False, shuffle: bool = True,
                 existing: np.ndarray | None = None):
    """A batch of ``k`` updates: ``k // 2`` deletions of uniformly chosen existing
    edges and ``k - k // 2`` insertions of uniform new edges (weights uniform in
    [1, wmax]).  For an undirected graph, ``src``/``dst`` list each edge once and
    every update is an unordered pair, emitted in a random orientation.

    Returns (bsrc, bdst, bw, bop) with op 0 = delete, 1 = insert.
    """
    m = src.size
    n_del = k // 2
    n_ins = k - n_del
    di = _distinct_indices(stream_seed(seed, "del"), m, n_del)
    ds = src[di].astype(np.int64)
    dd = dst[di].astype(np.int64)
    if existing is None:
        existing = edge_keys(src, dst, undirected)
    iu, iv = _new_pairs(seed, n, n_ins, existing, undirected)
    iw = uniform_int(stream_seed(seed, "ins_w"), 0, n_ins, 1, wmax)
    bsrc = np.concatenate([ds, iu])
    bdst = np.concatenate([dd, iv])
    bw = np.concatenate([np.zeros(n_del, np.int64), iw])
    bop = np.concatenate([np.zeros(n_del, np.uint8), np.ones(n_ins, np.uint8)])
    if undirected:
        flip = (draws(stream_seed(seed, "orient"), 0, k) & np.uint64(1)).astype(bool)
        bsrc, bdst = np.where(flip, bdst, bsrc), np.where(flip, bsrc, bdst)
    if shuffle and k > 0:
        perm = np.argsort(draws(stream_seed(seed, "perm"), 0, k), kind="stable")
        bsrc, bdst, bw, bop = bsrc[perm], bdst[perm], bw[perm], bop[perm]
    return (bsrc.astype(np.int32), bdst.astype(np.int32), bw.astype(np.int32),
            bop.astype(np.uint8))


def random_small_graph(n: int, m: int, seed: int, wmax: int = 20, undirected: bool = False):
    """Uniform random simple graph for small exhaustive tests: ``m`` distinct
    pairs (u != v) drawn uniformly.  Returns (src, dst, w)."""
    cap = n * (n - 1) // (2 if undirected else 1)
    m = min(m, cap)
    u, v = _new_pairs(seed, n, m, np.empty(0, np.int64), undirected)
    w = uniform_int(stream_seed(seed, "w"), 0, m, 1, wmax)
    return u.astype(np.int32), v.astype(np.int32), w.astype(np.int32)


# ----------------------------------------------------------------------------- workloads

def c1_workload(instance: int = 0):
    """Directed R-MAT, 2^14 vertices, 2^18 arcs, weights [1,100]; one batch of
    1 % of |E| (2,621 updates, half deletions)."""
    seed = config_seed(0, instance)
    n, s, d, w = rmat_directed(14, 1 << 18, seed)
    k = int(0.01 * s.size)
    batch = update_batch(n, s, d, k, seed + 1)
    return n, s, d, w, batch


def c2r_graph(scale: int = 22, instance: int = 0):
    """Directed R-MAT scale 22 (2^22 vertices, 16 * 2^22 arcs), weights [1,100]."""
    seed = config_seed(1, instance)
    return rmat_directed(scale, 16 << scale, seed)


def c2g_graph(side: int = 4096, instance: int = 0):
    """side x side 4-neighbour grid, weights [1,1000] per undirected edge."""
    seed = config_seed(1, 500 + instance)
    return grid4(side, side, seed, 1000)


def c3_graph(scale: int = 20, instance: int = 0):
    """Undirected R-MAT scale 20, average degree 32 (16 * 2^scale edges)."""
    seed = config_seed(2, instance)
    return rmat_undirected(scale, 16 << scale, seed)
