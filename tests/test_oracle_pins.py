"""Pins of the CPU oracle against what the mathematics and the paper fix.

None of these checks re-types the oracle's own formula: shortest paths are
checked against Floyd-Warshall and Bellman-Ford run here and against the
optimality conditions; PageRank against a dense linear solve, closed forms and
the normalisation identity; triangle counts against trace(A^3)/6, a brute
triple loop and closed forms; batch application against set properties.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = oracle.INF


# ------------------------------------------------------------------ helpers (independent)

def floyd_warshall(n, src, dst, w):
    big = np.int64(1) << 50
    D = np.full((n, n), big, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for a, b, c in zip(src, dst, w):
        D[a, b] = min(D[a, b], c)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def bellman_ford(n, src, dst, w, s):
    d = [math.inf] * n
    d[s] = 0
    for _ in range(n):
        changed = False
        for a, b, c in zip(src, dst, w):
            if d[a] + c < d[b]:
                d[b] = d[a] + c
                changed = True
        if not changed:
            break
    return [INF if x == math.inf else x for x in d]


def dense_pagerank(n, src, dst, d):
    """Solve (I - d S) pi = (1-d)/n 1, S column-stochastic with dangling columns
    replaced by the uniform vector (numpy.linalg.solve)."""
    outdeg = np.bincount(np.asarray(src, np.int64), minlength=n).astype(float)
    S = np.zeros((n, n))
    for a, b in zip(src, dst):
        S[b, a] += 1.0 / outdeg[a]
    for a in range(n):
        if outdeg[a] == 0:
            S[:, a] = 1.0 / n
    return np.linalg.solve(np.eye(n) - d * S, np.full(n, (1 - d) / n))


def dense_pagerank_dropped(n, src, dst, d):
    """The paper's iteration target with dangling mass dropped:
    (I - d P^T) x = (1-d)/n 1."""
    outdeg = np.bincount(np.asarray(src, np.int64), minlength=n).astype(float)
    P = np.zeros((n, n))
    for a, b in zip(src, dst):
        P[b, a] += 1.0 / outdeg[a]
    return np.linalg.solve(np.eye(n) - d * P, np.full(n, (1 - d) / n))


def trace_tc(n, u, v):
    A = np.zeros((n, n), dtype=np.int64)
    A[u, v] = 1
    A[v, u] = 1
    return int(np.trace(A @ A @ A) // 6)


def brute_tc(n, u, v):
    E = set()
    for a, b in zip(u, v):
        E.add((min(a, b), max(a, b)))
    c = 0
    for a, b, x in itertools.combinations(range(n), 3):
        if (a, b) in E and (b, x) in E and (a, x) in E:
            c += 1
    return c


def small_directed(n, m, seed, wmax=20):
    return graphgen.random_small_graph(n, m, seed, wmax)


# ------------------------------------------------------------------ SSSP

@pytest.mark.parametrize("seed", range(6))
def test_sssp_matches_floyd_warshall(seed):
    n = 48
    s, d, w = small_directed(n, 150 + 30 * seed, 100 + seed)
    D = floyd_warshall(n, s, d, w)
    for source in (0, 7, 31):
        got = oracle.sssp(n, s, d, w, source)
        want = np.where(D[source] >= (1 << 50), INF, D[source])
        assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(4))
def test_sssp_matches_bellman_ford(seed):
    n = 30
    s, d, w = small_directed(n, 90, 200 + seed, wmax=7)
    assert list(oracle.sssp(n, s, d, w, 3)) == bellman_ford(n, s, d, w, 3)


def check_sssp_invariants(n, s, d, w, source, dist):
    s = s.astype(np.int64); d = d.astype(np.int64); w = w.astype(np.int64)
    dist64 = dist.astype(np.int64)
    assert dist[source] == 0
    fin = dist64[s] < INF
    # no arc can still be relaxed
    assert np.all(dist64[d][fin] <= dist64[s][fin] + w[fin])
    # every reachable v != source has a tight in-arc
    tight = fin & (dist64[d] == dist64[s] + w)
    has_tight = np.zeros(n, bool)
    has_tight[d[tight]] = True
    reach = dist64 < INF
    reach[source] = False
    assert np.all(has_tight[reach])
    # INF exactly on the vertices a BFS cannot reach
    adj_off = np.zeros(n + 1, np.int64)
    np.add.at(adj_off, s + 1, 1)
    adj_off = np.cumsum(adj_off)
    order = np.argsort(s, kind="stable")
    col = d[order]
    seen = np.zeros(n, bool)
    seen[source] = True
    frontier = [source]
    while frontier:
        nxt = []
        for a in frontier:
            for b in col[adj_off[a]:adj_off[a + 1]]:
                if not seen[b]:
                    seen[b] = True
                    nxt.append(b)
        frontier = nxt
    assert np.array_equal(seen, dist < INF)


def test_sssp_invariants_rmat_after_batch():
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    s2, d2, w2, stats = oracle.apply(n, s, d, w, bs, bd, bw, bo)
    dist = oracle.sssp(n, s2, d2, w2, 0)
    check_sssp_invariants(n, s2, d2, w2, 0, dist)
    assert stats[0] == 1310 and stats[2] == 0  # every deletion hit an existing arc


def test_sssp_unreachable_and_isolated():
    # 0 -> 1 -> 2, 3 isolated, 4 -> 0 (4 unreachable from 0)
    s = np.array([0, 1, 4]); d = np.array([1, 2, 0]); w = np.array([5, 6, 1])
    assert list(oracle.sssp(5, s, d, w, 0)) == [0, 5, 11, INF, INF]
    assert list(oracle.sssp(1, [], [], [], 0)) == [0]


def test_sssp_fig_dynsssp_reconstructed():
    g = json.load(open(os.path.join(GOLDEN, "fig_dynsssp.json")))
    V = g["vertices"]
    e = np.array(g["edges"])
    b = np.array(g["batch"])
    before = oracle.sssp(g["n"], e[:, 0], e[:, 1], e[:, 2], g["source"])
    for name, val in g["printed_before"].items():
        assert before[V[name]] == val
    s2, d2, w2, _ = oracle.apply(g["n"], e[:, 0], e[:, 1], e[:, 2], b[:, 0], b[:, 1], b[:, 2], b[:, 3])
    after = oracle.sssp(g["n"], s2, d2, w2, g["source"])
    for name, val in g["printed_after"].items():
        assert after[V[name]] == val
    ins = b[b[:, 3] == 1]
    s3, d3, w3, _ = oracle.apply(g["n"], e[:, 0], e[:, 1], e[:, 2], ins[:, 0], ins[:, 1], ins[:, 2], ins[:, 3])
    mid = oracle.sssp(g["n"], s3, d3, w3, g["source"])
    assert mid[V["v"]] == 40 and mid[V["w"]] == 44 and mid[V["y"]] == before[V["y"]]


# ------------------------------------------------------------------ PageRank

@pytest.mark.parametrize("seed", range(6))
def test_pagerank_matches_dense_solve(seed):
    n = 40
    s, d, _ = small_directed(n, 60 + 25 * seed, 300 + seed)
    want = dense_pagerank(n, s, d, 0.85)
    got, it, conv = oracle.pagerank(n, s, d, 0.85, 1e-14, 5000)
    assert conv
    assert np.max(np.abs(got - want)) < 1e-12
    assert abs(got.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_pagerank_normalisation_identity(seed):
    """The dangling-uniform ranks equal x*/sum(x*) where x* solves the paper's
    dangling-dropped system x = (1-d)/n + d P^T x."""
    n = 36
    s, d, _ = small_directed(n, 50 + 20 * seed, 400 + seed)
    x = dense_pagerank_dropped(n, s, d, 0.85)
    got, _, _ = oracle.pagerank(n, s, d, 0.85, 1e-14, 5000)
    assert np.max(np.abs(got - x / x.sum())) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 5, 17])
def test_pagerank_closed_forms(n):
    # directed cycle, complete digraph and edgeless graph: all uniform
    cyc_s = np.arange(n); cyc_d = (np.arange(n) + 1) % n
    if n > 1:
        r, _, _ = oracle.pagerank(n, cyc_s, cyc_d, 0.85, 1e-14)
        assert np.allclose(r, 1.0 / n, atol=1e-14)
        pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
        ks, kd = np.array(pairs).T
        r, _, _ = oracle.pagerank(n, ks, kd, 0.85, 1e-14)
        assert np.allclose(r, 1.0 / n, atol=1e-14)
    r, it, _ = oracle.pagerank(n, [], [], 0.85, 1e-9)
    assert np.allclose(r, 1.0 / n, atol=1e-15)


def test_pagerank_two_vertices_by_hand():
    # 0 -> 1, vertex 1 dangling: pi0 = 1/(2+d), pi1 = (1+d)/(2+d)
    d = 0.85
    r, _, _ = oracle.pagerank(2, [0], [1], d, 1e-15)
    assert abs(r[0] - 1 / (2 + d)) < 1e-13 and abs(r[1] - (1 + d) / (2 + d)) < 1e-13


def test_pagerank_tolerance_bound():
    """At L1 step tol the Jacobi error is at most d/(1-d) * tol in L1."""
    n, s, d, w, _ = graphgen.c1_workload()
    tight, _, _ = oracle.pagerank(n, s, d, 0.85, 1e-14, 5000)
    loose, it, conv = oracle.pagerank(n, s, d, 0.85, 1e-9, 1000)
    assert conv and 5 < it < 400
    assert np.abs(loose - tight).sum() <= 0.85 / 0.15 * 1e-9 * 1.01 + 1e-13


# ------------------------------------------------------------------ triangle counting

@pytest.mark.parametrize("seed", range(6))
def test_tc_matches_trace(seed):
    n = 60 + 10 * seed
    u, v, _ = graphgen.random_small_graph(n, 300 + 80 * seed, 500 + seed, undirected=True)
    assert oracle.triangles(n, u, v) == trace_tc(n, u, v)


@pytest.mark.parametrize("seed", range(3))
def test_tc_matches_brute_triple_loop(seed):
    n = 30
    u, v, _ = graphgen.random_small_graph(n, 120, 600 + seed, undirected=True)
    # orientation of the pairs must not matter
    flip = np.arange(u.size) % 2 == 1
    u2, v2 = np.where(flip, v, u), np.where(flip, u, v)
    assert oracle.triangles(n, u2, v2) == brute_tc(n, u, v)


@pytest.mark.parametrize("n", range(3, 13))
def test_tc_closed_forms(n):
    pairs = np.array(list(itertools.combinations(range(n), 2)))
    assert oracle.triangles(n, pairs[:, 0], pairs[:, 1]) == math.comb(n, 3)
    cyc = np.arange(n)
    assert oracle.triangles(n, cyc, (cyc + 1) % n) == (1 if n == 3 else 0)
    if n >= 5:  # wheel: hub 0, rim 1..n-1 (r = n-1 >= 4 rim vertices) -> r triangles
        rim = np.arange(1, n)
        u = np.concatenate([np.zeros(n - 1, int), rim])
        v = np.concatenate([rim, np.roll(rim, -1)])
        assert oracle.triangles(n, u, v) == n - 1


def test_tc_grid_and_bipartite_zero():
    n, s, d, _ = graphgen.grid4(12, 9, 1)
    keep = s < d
    assert oracle.triangles(n, s[keep], d[keep]) == 0
    a, b = np.meshgrid(np.arange(5), np.arange(5, 11))
    assert oracle.triangles(11, a.ravel(), b.ravel()) == 0


def test_tc_insert_one_edge_adds_common_neighbours():
    n = 70
    u, v, _ = graphgen.random_small_graph(n, 500, 700, undirected=True)
    E = set(zip(np.minimum(u, v).tolist(), np.maximum(u, v).tolist()))
    nb = {x: set() for x in range(n)}
    for a, b in E:
        nb[a].add(b); nb[b].add(a)
    a, b = next((a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in E and nb[a] & nb[b])
    base = oracle.triangles(n, u, v)
    after = oracle.triangles(n, np.append(u, a), np.append(v, b))
    assert after - base == len(nb[a] & nb[b])


# ------------------------------------------------------------------ batch application

def _as_dict(s, d, w, undirected=False):
    out = {}
    for a, b, c in zip(s.tolist(), d.tolist(), w.tolist()):
        key = (min(a, b), max(a, b)) if undirected else (a, b)
        out[key] = c
    return out


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", range(5))
def test_apply_set_properties(seed, undirected):
    n = 50
    s, d, w = graphgen.random_small_graph(n, 300, 800 + seed, undirected=undirected)
    bs, bd, bw, bo = graphgen.update_batch(n, s, d, 120, 900 + seed, undirected=undirected)
    # add noise the generator never makes: repeats, a delete of an absent edge,
    # an insert of a present edge, and a delete + re-insert of one edge
    ex = (int(s[0]), int(d[0]))
    bs = np.concatenate([bs, bs[:10], [ex[0], ex[0], s[1]], [7]])
    bd = np.concatenate([bd, bd[:10], [ex[1], ex[1], d[1]], [8]])
    bw = np.concatenate([bw, bw[:10] + 1, [0, 99, 5], [3]])
    bo = np.concatenate([bo, bo[:10], [0, 1, 1], [0]]).astype(np.uint8)
    s2, d2, w2, stats = oracle.apply(n, s, d, w, bs, bd, bw, bo, undirected=undirected)
    old = _as_dict(s, d, w, undirected)
    new = _as_dict(s2, d2, w2, undirected)
    keys = [(min(a, b), max(a, b)) if undirected else (a, b) for a, b in zip(bs.tolist(), bd.tolist())]
    dels = {k for k, o in zip(keys, bo) if o == 0}
    ins = {}
    for k, o, c in zip(keys, bo, bw.tolist()):
        if o == 1:
            ins[k] = min(ins.get(k, 1 << 40), c)
    # sorted, simple, no self-loops, canonical orientation
    keys2 = list(zip(s2.tolist(), d2.tolist()))
    assert keys2 == sorted(set(keys2))
    assert all(a != b for a, b in keys2)
    if undirected:
        assert all(a < b for a, b in keys2)
    for k, c in old.items():
        if k not in dels:
            assert new[k] == c                      # untouched or ignored insert keeps weight
    for k in dels:
        if k not in ins:
            assert k not in new
    for k, c in ins.items():
        if k in old and k not in dels:
            assert new[k] == old[k]                 # B2
        else:
            assert new[k] == c                      # B4 / B5
    assert new[ex] == 99                            # deleted and re-inserted with weight 99
    assert len(new) == len(old) - stats[0] + stats[1]
    assert stats[2] == len([k for k in dels if k not in old])


def test_apply_roundtrip_and_rejects():
    n = 40
    s, d, w = graphgen.random_small_graph(n, 200, 42)
    _, _, _, (bs, bd, bw, bo) = (None, None, None, graphgen.update_batch(n, s, d, 60, 43))
    ins = bo == 1
    s2, d2, w2, _ = oracle.apply(n, s, d, w, bs[ins], bd[ins], bw[ins], bo[ins])
    back = oracle.apply(n, s2, d2, w2, bs[ins], bd[ins], bw[ins], np.zeros(ins.sum(), np.uint8))
    ref = oracle.apply(n, s, d, w, [], [], [], [])
    for x, y in zip(back[:3], ref[:3]):
        assert np.array_equal(x, y)
    for bad in ([(3, 3, 1, 1)], [(0, n, 1, 1)], [(-1, 2, 1, 0)], [(1, 2, 1, 2)], [(1, 2, -4, 1)], [(1, 2, 0, 1)]):
        b = np.array(bad)
        with pytest.raises(oracle.InvalidBatch):
            oracle.apply(n, s, d, w, b[:, 0], b[:, 1], b[:, 2], b[:, 3])


def test_symmetrise():
    s = np.array([0, 1, 2, 3, 1]); d = np.array([1, 0, 1, 0, 3])
    u, v = oracle.symmetrise(s, d)
    assert list(zip(u.tolist(), v.tolist())) == [(0, 1), (0, 3), (1, 2), (1, 3)]


# ------------------------------------------------------------------ random sequences

@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10_000), n=st.integers(2, 24), frac=st.floats(0.05, 0.6))
def test_random_batch_sequences_against_brute_force(seed, n, frac):
    m = max(1, int(frac * n * (n - 1)))
    s, d, w = graphgen.random_small_graph(n, m, seed, wmax=9)
    us, uv, _ = graphgen.random_small_graph(n, max(1, m // 2), seed + 1, undirected=True)
    for step in range(3):
        free = n * (n - 1) - s.size
        k = min(6, 2 * s.size, 2 * free)
        if k > 0:
            bs, bd, bw, bo = graphgen.update_batch(n, s, d, k, seed * 7 + step)
            s, d, w, _ = oracle.apply(n, s, d, w, bs, bd, bw, bo)
        free = n * (n - 1) // 2 - us.size
        k = min(6, 2 * us.size, 2 * free)
        if k > 0:
            bs, bd, bw, bo = graphgen.update_batch(n, us, uv, k, seed * 11 + step, undirected=True)
            us, uv, _, _ = oracle.apply(n, us, uv, None, bs, bd, bw, bo, undirected=True)
        D = floyd_warshall(n, s, d, w)
        want = np.where(D[0] >= (1 << 50), INF, D[0])
        assert np.array_equal(oracle.sssp(n, s, d, w, 0), want)
        assert oracle.triangles(n, us, uv) == trace_tc(n, us, uv)
        r, _, _ = oracle.pagerank(n, s, d, 0.85, 1e-14, 5000)
        assert np.max(np.abs(r - dense_pagerank(n, s, d, 0.85))) < 1e-11


# ------------------------------------------------------------------ generator

def test_generator_native_matches_numpy_definition():
    s1, d1 = graphgen._rmat_candidates(99, 11, 3, 4000, 0.57, 0.19, 0.19)
    s2, d2 = graphgen._rmat_candidates_fast(99, 11, 3, 4000, 0.57, 0.19, 0.19)
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    k = (s1 << 11) | d1
    assert np.array_equal(graphgen._first_unique(k, 2500), graphgen._first_unique_fast(k, 2500, 22))


def test_generator_shapes():
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    assert n == 16384 and s.size == 262144
    keys = (s.astype(np.int64) << 32) | d
    assert np.unique(keys).size == s.size and np.all(s != d)
    assert w.min() >= 1 and w.max() <= 100
    assert bs.size == 2621 and int((bo == 0).sum()) == 1310
    # R-MAT skew: vertex 0 is the largest hub
    assert np.bincount(s, minlength=n).argmax() == 0
