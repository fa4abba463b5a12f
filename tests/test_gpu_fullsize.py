"""GPU parity at the full benchmark sizes, in the configuration bench.py times.

* R-MAT scale 22 (4,194,304 vertices, 67,108,864 arcs), two 100k batches, with
  extrapolated (the bench's setting) and with plain Jacobi PageRank steps:
  distances bit-exact against the oracle's Dijkstra, the parent array a tight
  shortest-path tree, PageRank within max-abs 1e-10 of the oracle's power
  iteration.
* R-MAT scale 22 with four 1M-update batches (enough diff entries and
  tombstones to pass the merge threshold) and then one 10k batch: distances
  bit-exact, PageRank within max-abs 1e-10 of the oracle.
* 4096 x 4096 grid, one 100k batch, near-far SSSP (bucket width 8000):
  distances bit-exact against Dijkstra, PageRank within max-abs 1e-10 of the
  oracle's power iteration.
* Undirected R-MAT scale 20, batches of 0.1 %, 1 % and 5 % of the edges in a
  row: the maintained triangle count equals the oracle's count after each
  (stored in tests/golden/tc_rmat20.json by tests/golden/make_tc_rmat20.py, since
  a scale-20 recount takes minutes on one core) and the static forward count of
  the same graph.
* 4,096 R-MAT graphs (415 M arcs), one step: every member of a seeded sample of
  64, plus the largest, bit-exact against the oracle.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu

INF = dg.DG_INF


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def check_tree(n, s, d, w, src, dist, par):
    """Parents of reachable vertices are tight arcs of (s, d, w), sorted by (s, d)."""
    keys = (s.astype(np.int64) << 32) | d.astype(np.int64)
    assert np.all(keys[1:] > keys[:-1])
    reach = dist < INF
    assert dist[src] == 0 and par[src] == -1
    assert np.all(par[~reach] == -1)
    v = np.nonzero(reach)[0]
    v = v[v != src]
    q = (par[v].astype(np.int64) << 32) | v.astype(np.int64)
    pos = np.searchsorted(keys, q)
    assert np.all(pos < keys.size) and np.all(keys[np.minimum(pos, keys.size - 1)] == q)
    assert np.all(dist[par[v]].astype(np.int64) + w[pos] == dist[v].astype(np.int64))


def batches_for(n, s, d, k, config, count, wmax, undirected=False):
    keys = graphgen.edge_keys(s, d, undirected)
    return [graphgen.update_batch(n, s, d, k, graphgen.config_seed(config, 100 + i), wmax=wmax,
                                  undirected=undirected, existing=keys) for i in range(count)]


def bench_config(**kw):
    """The configuration bench.py runs: extrapolated PageRank steps, the rest default."""
    c = dg.Config()
    c.pr_extrapolate = 1
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_fullsize_rmat22_sssp_pagerank():
    """The bench's configuration (extrapolated PageRank steps) and plain Jacobi
    steps on the same batches, both against one oracle run."""
    t0 = time.perf_counter()
    n, s, d, w = graphgen.c2r_graph(22)
    bats = batches_for(n, s, d, 100000, 1, 2, 100)
    say("R-MAT 22 SSSP + PageRank, two 100k batches; inputs", round(time.perf_counter() - t0, 1), "s")
    got = {}
    for extrap in (1, 0):
        G = dg.Graph(n, s, d, w, config=bench_config(pr_extrapolate=extrap))
        qs = G.sssp_attach(0)
        qp = G.pr_attach(0.85, 1e-9, 1000)
        steps = 0
        for b in bats:
            st = G.apply(*b)
            steps += st.pr_iterations
        dist, par = qs.read()
        rank, _, conv = qp.read()
        G.close()
        say("extrapolated" if extrap else "plain", "PageRank steps over the batches", steps)
        got[extrap] = (dist, par, rank, conv)
    cs, cd, cw = s, d, w
    for b in bats:
        cs, cd, cw, ost = oracle.apply(n, cs, cd, cw, *b)
    say("oracle Dijkstra + power iteration at full size")
    want_d = oracle.sssp(n, cs, cd, cw, 0)
    want, _, oconv = oracle.pagerank(n, cs, cd, 0.85, 1e-9, 1000)
    assert oconv
    for extrap, (dist, par, rank, conv) in got.items():
        assert np.array_equal(dist, want_d)
        check_tree(n, cs, cd, cw, 0, dist, par)
        err = float(np.max(np.abs(rank - want)))
        say("extrapolated" if extrap else "plain", "PageRank max-abs vs oracle", err)
        assert conv and err <= 1e-10
        assert abs(float(rank.sum()) - 1.0) <= 1e-12


def test_fullsize_rmat22_large_batches_through_merge():
    t0 = time.perf_counter()
    n, s, d, w = graphgen.c2r_graph(22)
    keys = graphgen.edge_keys(s, d, False)
    bats = [graphgen.update_batch(n, s, d, k, graphgen.config_seed(1, 300 + i), wmax=100, existing=keys)
            for i, k in enumerate([1000000] * 4 + [10000])]
    say("R-MAT 22 SSSP + PageRank, four 1M batches and one 10k batch; inputs", round(time.perf_counter() - t0, 1), "s")
    G = dg.Graph(n, s, d, w, config=bench_config())
    qs = G.sssp_attach(0)
    qp = G.pr_attach(0.85, 1e-9, 1000)
    merged = 0
    for i, b in enumerate(bats):
        st = G.apply(*b)
        merged += st.merged
        say("batch", i, "k", b[0].size, "merged", st.merged, "diff", st.diff_entries, "tombstones", st.tombstones)
    assert merged >= 1
    dist, par = qs.read()
    rank, _, conv = qp.read()
    G.close()
    say("oracle: five edge-list applications, Dijkstra, power iteration")
    cs, cd, cw = s, d, w
    for b in bats:
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, *b)
    assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, 0))
    check_tree(n, cs, cd, cw, 0, dist, par)
    want, _, oconv = oracle.pagerank(n, cs, cd, 0.85, 1e-9, 1000)
    assert conv and oconv
    assert float(np.max(np.abs(rank - want))) <= 1e-10


def test_fullsize_grid_sssp_pagerank():
    t0 = time.perf_counter()
    n, s, d, w = graphgen.c2g_graph(4096)
    bats = batches_for(n, s, d, 100000, 1, 1, 1000)
    say("grid 4096^2 near-far SSSP + PageRank, one 100k batch; inputs", round(time.perf_counter() - t0, 1), "s")
    G = dg.Graph(n, s, d, w, config=bench_config(sssp_delta=8000))
    qs = G.sssp_attach(0)
    qp = G.pr_attach(0.85, 1e-9, 1000)
    G.apply(*bats[0])
    dist, par = qs.read()
    rank, _, conv = qp.read()
    G.close()
    cs, cd, cw, _ = oracle.apply(n, s, d, w, *bats[0])
    say("oracle Dijkstra and power iteration on the grid")
    assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, 0))
    check_tree(n, cs, cd, cw, 0, dist, par)
    want, _, oconv = oracle.pagerank(n, cs, cd, 0.85, 1e-9, 1000)
    err = float(np.max(np.abs(rank - want)))
    say("grid PageRank max-abs vs oracle", err)
    assert conv and oconv
    assert abs(float(rank.sum()) - 1.0) <= 1e-12
    assert err <= 1e-10


def test_fullsize_grid_pagerank_residual_push():
    """4096 x 4096 grid, one 10k batch, PageRank by residual push (pr_mode 3):
    within max-abs 1e-10 of the oracle's power iteration."""
    n, s, d, w = graphgen.c2g_graph(4096)
    b = batches_for(n, s, d, 10000, 1, 1, 1000)[0]
    say("grid 4096^2 PageRank residual push, one 10k batch")
    c = dg.Config()
    c.pr_mode = 3
    G = dg.Graph(n, s, d, w, config=c)
    qp = G.pr_attach(0.85, 1e-9, 1000)
    st = G.apply(*b)
    rank, it, conv = qp.read()
    G.close()
    say("push rounds", it, "arcs pushed", st.edges_traversed)
    cs, cd, cw, _ = oracle.apply(n, s, d, w, *b)
    want, _, oconv = oracle.pagerank(n, cs, cd, 0.85, 1e-9, 1000)
    err = float(np.max(np.abs(rank - want)))
    say("grid push PageRank max-abs vs oracle", err)
    assert conv and oconv and err <= 1e-10


def test_fullsize_tc_rmat20_against_golden_counts():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tc_rmat20.json")))
    t0 = time.perf_counter()
    n, s, d = graphgen.c3_graph(20)[:3]
    assert (n, s.size) == (gold["graph"]["vertices"], gold["graph"]["edges"])
    keys = graphgen.edge_keys(s, d, True)
    bats = [graphgen.update_batch(n, s, d, b["k"], b["seed"], undirected=True, existing=keys)
            for b in gold["batches"]]
    say("undirected R-MAT 20 TC, batches of 0.1 %, 1 % and 5 %; inputs", round(time.perf_counter() - t0, 1), "s")
    G = dg.Graph(n, s, d, None, undirected=True)
    q = G.tc_attach()
    assert q.read() == gold["counts"][0]
    for i, (b, want) in enumerate(zip(bats, gold["counts"][1:])):
        st = G.apply(*b)
        assert (st.deleted, st.inserted) == (gold["batches"][i]["deleted"], gold["batches"][i]["inserted"])
        dyn = q.read()
        say("batch", i, "k", b[0].size, "count", dyn, "want", want)
        assert dyn == want, i
        assert G.tc_static() == want, i
    G.close()


def test_tc_rmat17_against_oracle():
    n, s, d = graphgen.c3_graph(17)[:3]
    k = int(0.01 * s.size)
    bats = batches_for(n, s, d, k, 2, 2, 100, undirected=True)
    say("undirected R-MAT 17 TC against the oracle, two 1 % batches")
    G = dg.Graph(n, s, d, None, undirected=True)
    q = G.tc_attach()
    cs, cd = s, d
    for b in bats:
        G.apply(*b)
        cs, cd, _, _ = oracle.apply(n, cs, cd, np.ones(cs.size, np.int32), *b, undirected=True)
    assert q.read() == oracle.triangles(n, cs, cd)
    G.close()


def test_fullsize_batched4096_sssp_sample():
    t0 = time.perf_counter()
    count = 4096
    seed = graphgen.config_seed(3, 0)
    scales = graphgen.uniform_int(graphgen.stream_seed(seed, "scale"), 0, count, 10, 14)
    frac = 0.01 + 0.09 * graphgen.uniform01(graphgen.stream_seed(seed, "frac"), 0, count)
    members, bats = [], []
    for i in range(count):
        sc = int(scales[i])
        n, s, d, w = graphgen.rmat_directed(sc, 16 << sc, graphgen.config_seed(3, i))
        members.append((n, s, d, w))
        k = int(frac[i] * (16 << sc))
        bats.append(graphgen.update_batch(n, s, d, k, graphgen.config_seed(3, 100000 + i),
                                          existing=graphgen.edge_keys(s, d, False)))
    say("batched set of", count, "R-MAT graphs, one step; inputs", round(time.perf_counter() - t0, 1), "s")
    S = dg.GraphSet(members)  # captured frontier rounds, the set's default
    info = S.info()
    assert info["count"] == count and info["arcs"] == sum(m[1].size for m in members)
    S.sssp_attach(np.zeros(count, np.int32))
    st = S.apply(bats)
    assert st.updates == sum(b[0].size for b in bats)
    pick = graphgen.uniform_int(graphgen.stream_seed(seed, 991), 0, 64, 0, count - 1).tolist()
    pick.append(int(np.argmax([m[0] for m in members])))
    for i in sorted(set(pick)):
        n, s, d, w = members[i]
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *bats[i])
        dist, par = S.read(i)
        assert np.array_equal(dist, oracle.sssp(n, s2, d2, w2, 0)), i
        check_tree(n, s2, d2, w2, 0, dist, par)
    S.close()
