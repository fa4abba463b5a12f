"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Shortest-path distances, exported edge sets and triangle counts must be
bit-exact; PageRank must be within max-abs 1e-10 of the oracle run at the same
L1 tolerance (1e-9).  Parent arrays are checked for validity (several shortest
path trees are correct).  Every case prints its name and seed first so that a
failing run names it.
"""
import json
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu

INF = dg.DG_INF
PR_TOL = 1e-9
PR_MAXABS = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def cfg(merge=0.0, heavy=0, tol_scale=0.0, persistent=0, delta=0):
    c = dg.Config()
    c.merge_threshold = merge
    c.heavy_degree = heavy
    c.pr_tol_scale = tol_scale
    c.sssp_persistent = persistent
    c.sssp_delta = delta
    return c


def assert_edges(G, s, d, w, undirected=False):
    gs, gd, gw = G.export()
    assert gs.size == s.size
    assert np.array_equal(gs, s) and np.array_equal(gd, d)
    if not undirected:
        assert np.array_equal(gw, w)


def assert_tree(n, s, d, w, source, dist, parent):
    """parent[] is a shortest-path tree of the distances dist[]."""
    emap = {}
    for a, b, c in zip(s.tolist(), d.tolist(), w.tolist()):
        emap[(a, b)] = c
    assert parent[source] == -1
    for v in range(n):
        if v == source:
            continue
        if dist[v] >= INF:
            assert parent[v] == -1
            continue
        p = int(parent[v])
        assert (p, v) in emap, (p, v)
        assert int(dist[p]) + emap[(p, v)] == int(dist[v])


def rmat_small(scale=12, deg=16, seed=7):
    return graphgen.rmat_directed(scale, deg << scale, seed)


# ------------------------------------------------------------------ graph store

def test_build_and_export_c1():
    n, s, d, w, _ = graphgen.c1_workload()
    say("build/export C1")
    G = dg.Graph(n, s, d, w)
    os_, od, ow, _ = oracle.apply(n, s, d, w, [], [], [], [])
    assert_edges(G, os_, od, ow)
    assert G.info()["m"] == s.size


def test_diffcsr_figure_example():
    """Section 3.5 diff-CSR example (figure reconstructed from the printed array
    entries): deleting B->D leaves a tombstone, inserting E->C goes to the diff."""
    say("diff-CSR figure example")
    A, B, C, D, E, F = range(6)
    s = np.array([A, B, B, C, D, E, F]); d = np.array([B, C, D, A, E, F, D])
    G = dg.Graph(6, s, d, None, config=cfg(merge=1e9))
    G.apply([B, E], [D, C], [0, 1], [0, 1])
    info = G.info()
    assert info["tombstones"] == 1 and info["diff_entries"] == 1 and info["m"] == 7
    es, ed, _ = G.export()
    assert list(zip(es.tolist(), ed.tolist())) == sorted([(A, B), (B, C), (C, A), (D, E), (E, C), (E, F), (F, D)])


@pytest.mark.parametrize("diff_only", [0, 1])
def test_diffcsr_figure_vacancy(diff_only):
    """Section 3.5 example continued: after B->D left a tombstone, a later insert of
    B->E takes that vacant slot (B's row stays sorted: C, E) instead of the diff;
    with diff_only the diff level takes it."""
    say("diff-CSR figure example, vacancy reuse, diff_only", diff_only)
    A, B, C, D, E, F = range(6)
    s = np.array([A, B, B, C, D, E, F]); d = np.array([B, C, D, A, E, F, D])
    c = cfg(merge=1e9)
    c.diff_only = diff_only
    c.vertex_order = 1  # keep the figure's ids, so B's row is the figure's
    G = dg.Graph(6, s, d, None, config=c)
    G.apply([B, E], [D, C], [0, 1], [0, 1])
    G.apply([B], [E], [4], [1])
    info = G.info()
    if diff_only:
        assert info["tombstones"] == 1 and info["diff_entries"] == 2
    else:
        assert info["tombstones"] == 0 and info["diff_entries"] == 1
    es, ed, ew = G.export()
    want = sorted([(A, B), (B, C), (B, E), (C, A), (D, E), (E, C), (E, F), (F, D)])
    assert list(zip(es.tolist(), ed.tolist())) == want
    assert ew[want.index((B, E))] == 4
    q = G.sssp_attach(A)
    assert q.read()[0].tolist() == oracle.sssp(6, es, ed, ew, A).tolist()
    G.close()


@pytest.mark.parametrize("undirected", [False, True])
def test_vacancy_reuse_matches_diff_only(undirected):
    """Batches on graphs full of tombstones (no merges): new edges fill vacant
    slots next to their sorted positions.  The edge set, SSSP, PageRank and triangle
    counts equal the oracle after every batch, the diff level stays smaller than
    with diff_only, and tombstones + diff entries add up the same way."""
    say("vacancy reuse vs diff_only, undirected", undirected)
    if undirected:
        n, u, v = graphgen.rmat_undirected(11, 8 << 11, graphgen.config_seed(2, 70))
        s, d, w = u, v, None
    else:
        n, s, d, w = rmat_small(11, 16, 70)
    runs = {}
    for diff_only in (0, 1):
        c = cfg(merge=1e9)
        c.diff_only = diff_only
        G = dg.Graph(n, s, d, w, undirected=undirected, config=c)
        qt = G.tc_attach() if undirected else None
        qs = None if undirected else G.sssp_attach(0)
        qp = None if undirected else G.pr_attach(0.85, PR_TOL, 1000)
        cs, cd, cw = s, d, (w if w is not None else np.ones(s.size, np.int32))
        infos = []
        for i, k in enumerate([3000, 2000, 4000, 1000]):
            b = graphgen.update_batch(n, cs, cd, k, graphgen.config_seed(0, 700 + i), undirected=undirected)
            st = G.apply(*b)
            cs, cd, cw, ost = oracle.apply(n, cs, cd, cw, *b, undirected=undirected)
            assert (st.deleted, st.inserted) == (ost[0], ost[1])
            infos.append(G.info())
            es, ed, ew = G.export()
            assert np.array_equal(es, cs) and np.array_equal(ed, cd)
            if not undirected:
                assert np.array_equal(ew, cw)
                assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0))
                want, _, _ = oracle.pagerank(n, cs, cd, 0.85, PR_TOL, 1000)
                assert float(np.max(np.abs(qp.read()[0] - want))) <= PR_MAXABS
            else:
                assert qt.read() == oracle.triangles(n, cs, cd)
        runs[diff_only] = infos
        G.close()
    filled = 0
    for a, b in zip(runs[0], runs[1]):
        assert a["m"] == b["m"]
        # a filled vacancy is one tombstone fewer and one diff entry fewer
        assert a["tombstones"] + a["diff_entries"] <= b["tombstones"] + b["diff_entries"]
        assert b["tombstones"] - a["tombstones"] == b["diff_entries"] - a["diff_entries"]
        filled = b["diff_entries"] - a["diff_entries"]
    assert filled > 0


@pytest.mark.parametrize("diff_only", [0, 1])
def test_reinsert_after_reverse_vacancy_taken(diff_only):
    """Directed graph: u->v is deleted (tombstones in u's forward row and v's
    reverse row), then w->v takes v's reverse vacancy (w sits next to u in v's
    row), then u->v is inserted again: its forward tombstone is revived while its
    reverse slot is gone, so the reverse store takes it as a new arc.  A merge then
    rebuilds both directions; the edge set, SSSP and PageRank equal the oracle.
    (A serving run of batches followed by their inverses met this case.)"""
    say("re-insert after the reverse vacancy was taken, diff_only", diff_only)
    n = 64
    rng = np.random.default_rng(5)
    pairs = set()
    while len(pairs) < 400:
        a, b = int(rng.integers(0, n)), int(rng.integers(0, n))
        if a != b:
            pairs.add((a, b))
    pairs.discard((11, 40))
    pairs |= {(10, 40), (12, 40), (10, 41)}
    s = np.array([p[0] for p in sorted(pairs)], np.int32)
    d = np.array([p[1] for p in sorted(pairs)], np.int32)
    w = rng.integers(1, 50, size=s.size).astype(np.int32)
    c = cfg(merge=1e9)
    c.diff_only = diff_only
    c.vertex_order = 1
    G = dg.Graph(n, s, d, w, config=c)
    qs = G.sssp_attach(10)
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    cs, cd, cw = s, d, w
    steps = [
        ([10], [40], [0], [0]),          # delete 10->40: vacancies at 10's row and at 40's reverse row
        ([11], [40], [7], [1]),          # 11->40 is new; in 40's reverse row 11 sits right after 10
        ([10, 3], [40, 9], [5, 2], [1, 1]),  # 10->40 again: forward revive, reverse slot taken
    ]
    for b in steps:
        b = tuple(np.asarray(x, dt) for x, dt in zip(b, (np.int32, np.int32, np.int32, np.uint8)))
        G.apply(*b)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, *b)
        assert_edges(G, cs, cd, cw)
    G.merge()
    assert_edges(G, cs, cd, cw)
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 10))
    want, _, _ = oracle.pagerank(n, cs, cd, 0.85, PR_TOL, 1000)
    assert float(np.max(np.abs(qp.read()[0] - want))) <= PR_MAXABS
    # and a longer run of batches followed by their exact inverses, with merges
    m0 = G.info()["m"]
    for i in range(6):
        b = graphgen.update_batch(n, cs, cd, 60, graphgen.config_seed(0, 900 + i))
        dels = b[3] == 0
        keys = (cs.astype(np.int64) << 32) | cd
        pos = np.searchsorted(keys, (b[0][dels].astype(np.int64) << 32) | b[1][dels])
        inv_w = np.zeros(b[0].size, np.int32)
        inv_w[dels] = cw[pos]
        inv = (b[0], b[1], inv_w, dels.astype(np.uint8))
        for bb in (b, inv):
            G.apply(*bb)
            cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, *bb)
            assert_edges(G, cs, cd, cw)
        if i == 3:
            G.merge()
    assert G.info()["m"] == m0
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 10))
    G.close()


@pytest.mark.parametrize("merge", [0.0, -1.0, 1e9])
def test_batch_sequence_matches_oracle(merge):
    n, s, d, w = rmat_small(11, 16, 21)
    say("batch sequence merge", merge)
    G = dg.Graph(n, s, d, w, config=cfg(merge=merge))
    cs, cd, cw = s, d, w
    sizes = [1, 7, 100, 2000, 33, 640, 5000, 1, 0, 300, 1200, 9000]
    for i, k in enumerate(sizes):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 1000 + i)
        if i % 3 == 1 and k > 4:  # noise: repeats, absent deletes, present inserts
            bs = np.concatenate([bs, bs[:4], cd[:3], [cs[5]]]).astype(np.int32)
            bd = np.concatenate([bd, bd[:4], cs[:3], [cd[5]]]).astype(np.int32)
            bw = np.concatenate([bw, bw[:4] + 3, [7, 7, 7], [2]]).astype(np.int32)
            bo = np.concatenate([bo, bo[:4], [0, 0, 0], [1]]).astype(np.uint8)
        st = G.apply(bs, bd, bw, bo)
        cs, cd, cw, ost = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        assert (st.deleted, st.inserted) == (ost[0], ost[1]), (i, st.as_dict(), ost)
        assert_edges(G, cs, cd, cw)


def test_delete_then_reinsert_and_revive():
    n, s, d, w = rmat_small(9, 8, 5)
    say("delete + reinsert")
    G = dg.Graph(n, s, d, w, config=cfg(merge=1e9))
    # batch 1: delete 50 edges; batch 2: re-insert 25 of them with new weights and
    # delete+insert 10 others in the same batch
    k = 50
    G.apply(s[:k], d[:k], w[:k], np.zeros(k, np.uint8))
    cs, cd, cw, _ = oracle.apply(n, s, d, w, s[:k], d[:k], w[:k], np.zeros(k, np.uint8))
    bs = np.concatenate([s[:25], s[100:110], s[100:110]])
    bd = np.concatenate([d[:25], d[100:110], d[100:110]])
    bw = np.concatenate([np.full(25, 77), np.zeros(10), np.full(10, 55)]).astype(np.int32)
    bo = np.concatenate([np.ones(25), np.zeros(10), np.ones(10)]).astype(np.uint8)
    st = G.apply(bs, bd, bw, bo)
    cs, cd, cw, ost = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
    assert (st.deleted, st.inserted) == (ost[0], ost[1])
    assert_edges(G, cs, cd, cw)
    assert G.info()["tombstones"] == 25


def test_invalid_batch_changes_nothing():
    n, s, d, w = rmat_small(9, 8, 6)
    say("invalid batch")
    G = dg.Graph(n, s, d, w)
    q = G.sssp_attach(0)
    before = G.export()
    dist0, _ = q.read()
    for bad in ([(1, 1, 1, 1)], [(0, n, 1, 1)], [(2, 3, 1, 9)], [(2, 3, -5, 1)]):
        b = np.array(bad + [(s[0], d[0], 0, 0)], dtype=np.int64)
        with pytest.raises(dg.DGError) as e:
            G.apply(b[:, 0], b[:, 1], b[:, 2], b[:, 3])
        assert e.value.code == dg.DG_EINVAL
    after = G.export()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert np.array_equal(q.read()[0], dist0)


def test_build_rejects_bad_edge_lists():
    say("bad edge lists")
    for s, d in (([0, 1], [1, 1]), ([0, 0], [1, 1]), ([0, 5], [1, 2])):
        with pytest.raises(dg.DGError):
            dg.Graph(4, s, d)


# ------------------------------------------------------------------ SSSP

@pytest.mark.parametrize("heavy,persistent", [(0, 0), (8, 0), (1 << 20, 0), (0, 1), (8, 1), (0, 2), (8, 2), (0, 3),
                                             (8, 3)])
def test_sssp_c1_dynamic(heavy, persistent):
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("sssp C1 heavy", heavy, "persistent", persistent)
    G = dg.Graph(n, s, d, w, config=cfg(heavy=heavy, persistent=persistent))
    q = G.sssp_attach(0)
    dist, par = q.read()
    assert np.array_equal(dist, oracle.sssp(n, s, d, w, 0))
    G.apply(bs, bd, bw, bo)
    cs, cd, cw, _ = oracle.apply(n, s, d, w, bs, bd, bw, bo)
    want = oracle.sssp(n, cs, cd, cw, 0)
    dist, par = q.read()
    assert np.array_equal(dist, want)
    assert_tree(n, cs, cd, cw, 0, dist, par)
    sd, sp = G.sssp_static(0)
    assert np.array_equal(sd, want)
    assert_tree(n, cs, cd, cw, 0, sd, sp)


@pytest.mark.parametrize("persistent,delta", [(0, 0), (1, 0), (0, 15), (2, 0), (2, 15), (3, 0)])
def test_sssp_many_batches_with_merges(persistent, delta):
    n, s, d, w = rmat_small(12, 8, 33)
    say("sssp sequence persistent", persistent, "delta", delta)
    G = dg.Graph(n, s, d, w, config=cfg(merge=0.02, persistent=persistent, delta=delta))
    qs = [G.sssp_attach(0), G.sssp_attach(17)]
    cs, cd, cw = s, d, w
    merges = 0
    for i in range(22):
        k = [50, 400, 3, 1500][i % 4]
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 3000 + i)
        if i % 5 == 0:  # delete tree edges near the source on purpose
            dist, par = qs[0].read()
            kids = np.nonzero(par == 0)[0][:20]
            bs = np.concatenate([bs, np.zeros(kids.size, np.int32)]).astype(np.int32)
            bd = np.concatenate([bd, kids]).astype(np.int32)
            bw = np.concatenate([bw, np.zeros(kids.size, np.int32)]).astype(np.int32)
            bo = np.concatenate([bo, np.zeros(kids.size, np.uint8)]).astype(np.uint8)
        st = G.apply(bs, bd, bw, bo)
        merges += st.merged
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        for q, src in zip(qs, (0, 17)):
            dist, par = q.read()
            assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, src)), (i, src)
            if i % 7 == 0:
                assert_tree(n, cs, cd, cw, src, dist, par)
    assert merges >= 2


@pytest.mark.parametrize("persistent,delta", [(0, 0), (1, 0), (0, 1), (0, 700), (0, 6000), (2, 0), (2, 1), (2, 700),
                                            (3, 700)])
def test_sssp_grid_and_hub(persistent, delta):
    """High-diameter grid (many frontier steps) plus a hub above the heavy limit."""
    n, s, d, w = graphgen.grid4(40, 40, 9, 1000)
    hub = 5
    extra = np.setdiff1d(np.arange(0, n, 2), np.concatenate([[hub], d[s == hub]]))
    s = np.concatenate([s, np.full(extra.size, hub)]).astype(np.int32)
    d = np.concatenate([d, extra]).astype(np.int32)
    w = np.concatenate([w, np.full(extra.size, 5000)]).astype(np.int32)
    say("sssp grid+hub persistent", persistent, "delta", delta)
    G = dg.Graph(n, s, d, w, config=cfg(heavy=64, persistent=persistent, delta=delta))
    q = G.sssp_attach(0)
    dist, _ = q.read()
    assert np.array_equal(dist, oracle.sssp(n, s, d, w, 0))
    cs, cd, cw = s, d, w
    for i in range(6):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, 60, 4000 + i, wmax=1000)
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        dist, par = q.read()
        assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, 0))
        assert_tree(n, cs, cd, cw, 0, dist, par)


@pytest.mark.parametrize("delta", [0, 40])
def test_sssp_row_grows_past_heavy_limit(delta):
    """Frontier steps skip the chunk kernel while the graph's longest-row bound
    (set at build, raised by rows that gain diff entries, brought to the host with
    the counters) is within heavy_degree.  Batches that grow one row of a 30 x 30
    grid far past the limit are relaxed by steps that still see the old bound (the
    row walked in place by one wave) and then by chunked steps.  Distances equal
    the oracle's and the trees are valid after every batch."""
    n, s, d, w = graphgen.grid4(30, 30, 3, 50)
    say("sssp row grows past the heavy limit, delta", delta)
    G = dg.Graph(n, s, d, w, config=cfg(heavy=32, delta=delta))
    q = G.sssp_attach(0)
    assert np.array_equal(q.read()[0], oracle.sssp(n, s, d, w, 0))
    cs, cd, cw = s, d, w
    rng = np.random.default_rng(11)
    for i, hub in enumerate([1, 1, 450]):
        existing = set(zip(cs.tolist(), cd.tolist()))
        cand = [v for v in rng.permutation(n).tolist() if v != hub and (hub, v) not in existing][:300]
        bs = np.full(len(cand), hub, np.int32)
        bd = np.array(cand, np.int32)
        bw = rng.integers(1, 50, len(cand)).astype(np.int32)
        bo = np.ones(len(cand), np.uint8)
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        dist, par = q.read()
        assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, 0)), i
        assert_tree(n, cs, cd, cw, 0, dist, par)


def test_work_queue_refuses_deep_graphs():
    """The work-queue schedule refuses a graph whose breadth-first levels from the
    source pass 64 (a 100 x 100 grid: 198 levels) before its queue runs; the
    frontier schedules solve the same graph."""
    n, s, d, w = graphgen.grid4(100, 100, 9, 1000)
    say("work queue guard on a 100x100 grid")
    G = dg.Graph(n, s, d, w, config=cfg(persistent=1))
    with pytest.raises(dg.DGError) as e:
        G.sssp_attach(0)
    assert e.value.code == dg.DG_EINVAL and "64 hops" in str(e.value)
    G.close()
    G = dg.Graph(n, s, d, w, config=cfg(persistent=0, delta=3000))
    q = G.sssp_attach(0)
    assert np.array_equal(q.read()[0], oracle.sssp(n, s, d, w, 0))
    G.close()


@pytest.mark.parametrize("kind,delta", [("rmat", 0), ("rmat", 40), ("grid", 0), ("grid", 700)])
def test_sssp_rounds_captured_on_a_stream(kind, delta):
    """Frontier rounds (near-far rounds when delta > 0) captured into hipGraphs on a
    non-null stream and replayed for every batch; on the grid the walks and the
    relaxation run far past one graph's rounds, so the continuation graphs are
    replayed until the device-side counts are zero."""
    import torch

    if kind == "rmat":
        n, s, d, w = rmat_small(12, 8, 35)
    else:
        n, s, d, w = graphgen.grid4(48, 48, 21, 1000)
    say("sssp captured rounds on a stream", kind, "delta", delta)
    G = dg.Graph(n, s, d, w, config=cfg(persistent=2, delta=delta))
    stream = torch.cuda.Stream()
    G.set_stream(stream.cuda_stream)
    q = G.sssp_attach(0)
    cs, cd, cw = s, d, w
    for i in range(8):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, [40, 900, 5, 3000][i % 4], 5100 + i)
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        dist, par = q.read()
        assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, 0)), i
    assert_tree(n, cs, cd, cw, 0, dist, par)
    torch.cuda.synchronize()


def test_sssp_fig_dynsssp_reconstructed():
    g = json.load(open(os.path.join(GOLDEN, "fig_dynsssp.json")))
    say("fig dynsssp")
    e = np.array(g["edges"]); b = np.array(g["batch"]); V = g["vertices"]
    G = dg.Graph(g["n"], e[:, 0], e[:, 1], e[:, 2])
    q = G.sssp_attach(g["source"])
    dist, _ = q.read()
    for name, val in g["printed_before"].items():
        assert dist[V[name]] == val
    G.apply(b[:, 0], b[:, 1], b[:, 2], b[:, 3])
    dist, _ = q.read()
    for name, val in g["printed_after"].items():
        assert dist[V[name]] == val


def test_sssp_distance_saturates_at_inf():
    """A vertex whose shortest distance is INF or more reads as unreachable
    (INF, parent -1); every other distance stays exact.  Hand-computed: the only
    path to 1 weighs 2^30 - 1 = INF; 3 is reached through 2 at 5 + (2^30 - 10)."""
    W = (1 << 30) - 1
    s = [0, 0, 2, 1, 3, 2]
    d = [1, 2, 3, 3, 4, 5]
    w = [W, 5, (1 << 30) - 10, 1, 1, 7]
    say("sssp saturation at INF")
    for order in (0, 1):
        c = cfg()
        c.vertex_order = order
        G = dg.Graph(6, s, d, w, config=c)
        q = G.sssp_attach(0)
        want = np.array([0, INF, 5, (1 << 30) - 5, (1 << 30) - 4, 12], np.int32)
        dist, par = q.read()
        assert np.array_equal(dist, want)
        assert par.tolist() == [-1, -1, 0, 2, 3, 2]
        # without 0->2, every path to 2..5 weighs INF or more (3 and 4 through 1)
        G.apply([0], [2], [0], [0])
        dist, par = q.read()
        assert dist.tolist() == [0, INF, INF, INF, INF, INF]
        assert par.tolist() == [-1] * 6
        # 0->1 deleted and re-inserted with weight 3 in one batch: 1, 3, 4 come back
        G.apply([0, 0], [1, 1], [0, 3], [0, 1])
        dist, par = q.read()
        assert dist.tolist() == [0, 3, INF, 4, 5, INF]
        assert par.tolist() == [-1, 0, -1, 1, 3, -1]
        G.close()


def test_sssp_unreachable_and_disconnect():
    say("sssp disconnect")
    # chain 0->1->2->3, 4 isolated; delete 1->2 cuts 2 and 3
    G = dg.Graph(5, [0, 1, 2], [1, 2, 3], [1, 1, 1])
    q = G.sssp_attach(0)
    G.apply([1], [2], [0], [0])
    dist, par = q.read()
    assert list(dist) == [0, 1, INF, INF, INF] and list(par) == [-1, 0, -1, -1, -1]
    G.apply([0], [3], [9], [1])
    dist, par = q.read()
    assert list(dist) == [0, 1, INF, 9, INF] and par[3] == 0


# ------------------------------------------------------------------ PageRank

def pr_check(got, n, s, d):
    want, _, conv = oracle.pagerank(n, s, d, 0.85, PR_TOL, 1000)
    tight, _, _ = oracle.pagerank(n, s, d, 0.85, 1e-14, 5000)
    err = float(np.max(np.abs(got - want)))
    err_t = float(np.max(np.abs(got - tight)))
    print(f"    pr max-abs vs oracle@1e-9 {err:.3e}, vs oracle@1e-14 {err_t:.3e}", flush=True)
    assert conv
    assert abs(got.sum() - 1.0) < 1e-12
    assert err <= PR_MAXABS


@pytest.mark.parametrize("heavy,mode", [(0, 0), (8, 0), (0, 1), (0, 2), (8, 1)])
def test_pagerank_c1_dynamic(heavy, mode):
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("pagerank C1 heavy", heavy, "mode", mode)
    c = cfg(heavy=heavy)
    c.pr_mode = mode
    G = dg.Graph(n, s, d, w, config=c)
    q = G.pr_attach(0.85, PR_TOL, 1000)
    r, it, conv = q.read()
    pr_check(r, n, s, d)
    cs, cd, cw = s, d, w
    for i in range(4):
        if i:
            bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, [300, 5000, 20][i - 1], 5000 + i)
        st = G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        r, it, conv = q.read()
        assert conv and st.pr_affected > 0
        pr_check(r, n, cs, cd)
    rs, _ = G.pr_static(0.85, PR_TOL, 1000)
    pr_check(rs, n, cs, cd)


def hub_graph(n=1 << 14, hub_in=12000, seed=11):
    """Uniform arcs among the lower half of the vertices (the upper half is
    isolated) plus one hub with `hub_in` in-arcs, so that whole-graph pulls see
    rows far longer than a tile, runs of empty rows and tiny rows."""
    rng_s = graphgen.uniform_int(seed, 0, 80000, 0, n // 2 - 1)
    rng_d = graphgen.uniform_int(seed + 1, 0, 80000, 0, n // 2 - 1)
    hs = np.arange(1, hub_in + 1)
    src = np.concatenate([rng_s, hs])
    dst = np.concatenate([rng_d, np.full(hub_in, 0)])
    keep = src != dst
    key = np.unique((src[keep].astype(np.int64) << 32) | dst[keep].astype(np.int64))
    s = (key >> 32).astype(np.int32)
    d = (key & 0xFFFFFFFF).astype(np.int32)
    w = graphgen.uniform_int(seed + 2, 0, s.size, 1, 100).astype(np.int32)
    return n, s, d, w


@pytest.mark.parametrize("pull,tile", [(0, 0), (1, 0), (2, 0), (0, 1024), (0, 4096)])
def test_pagerank_whole_graph_pull(pull, tile):
    """Static solve and global-form updates, merge-path tiles with non-temporal
    streams (0), per-vertex waves (1) or tiles without the hints (2), with a live
    diff level (no merges), against the oracle."""
    n, s, d, w = hub_graph()
    say("pagerank whole-graph pull", pull, "arcs", s.size)
    c = cfg(merge=1e9)
    c.pr_mode = 2
    c.pr_pull = pull
    c.pr_tile = tile
    G = dg.Graph(n, s, d, w, config=c)
    q = G.pr_attach(0.85, PR_TOL, 1000)
    r, it, conv = q.read()
    pr_check(r, n, s, d)
    cs, cd, cw = s, d, w
    for i, k in enumerate([2000, 9000, 400]):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 7100 + i)
        # extra arcs into the hub so the diff level holds a long row too
        lo = 13000 + 600 * i
        extra_s = np.arange(lo, lo + 500, dtype=np.int32)
        bs = np.concatenate([bs, extra_s]); bd = np.concatenate([bd, np.zeros(500, np.int32)])
        bw = np.concatenate([bw, np.full(500, 3, np.int32)]); bo = np.concatenate([bo, np.ones(500, np.uint8)])
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        r, it, conv = q.read()
        assert conv
        pr_check(r, n, cs, cd)
    assert G.info()["diff_entries"] > 0
    rs, _ = G.pr_static(0.85, PR_TOL, 1000)
    pr_check(rs, n, cs, cd)


@pytest.mark.parametrize("kind,mode,pull", [("rmat", 2, 0), ("rmat", 2, 1), ("rmat", 1, 0), ("rmat", 0, 0),
                                            ("grid", 2, 0), ("grid", 1, 0)])
def test_pagerank_extrapolated_steps(kind, mode, pull):
    """Extrapolated Jacobi steps (pr_extrapolate = 1) against plain ones: both
    reach the oracle's ranks after the static solve and after every batch (global
    form over tiles or vertex waves, the local form on the affected set, automatic
    choice), and the extrapolated runs take no more steps in total.  R-MAT scale
    13 with uniform insertions has a slow, steady error mode for the move to
    remove; the grid is bipartite (eigenvalues near -d as well as +d), where a
    move taken on the L1 step ratio alone diverges and the one-step fit never
    lines up: there the fit against the step before the previous one (two-step
    moves) must take at most 70 % of the plain steps, with moves reported by the
    batches."""
    if kind == "rmat":
        n, s, d, w = rmat_small(scale=13)
    else:
        n, s, d, w = graphgen.grid4(48, 48, 5)
    say("pagerank extrapolated vs plain,", kind, "mode", mode, "pull", pull)
    steps = {}
    for extrap in (1, 0):
        c = cfg()
        c.pr_mode = mode
        c.pr_pull = pull
        c.pr_extrapolate = extrap
        G = dg.Graph(n, s, d, w, config=c)
        q = G.pr_attach(0.85, PR_TOL, 1000)
        r, it, conv = q.read()
        assert conv
        pr_check(r, n, s, d)
        total = it
        moves = 0
        cs, cd, cw = s, d, w
        for i, k in enumerate([40, 3000, 12000] if kind == "rmat" else [6, 200, 900]):
            bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 7700 + i)
            moves += G.apply(bs, bd, bw, bo).pr_moves
            cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
            r, it, conv = q.read()
            assert conv
            pr_check(r, n, cs, cd)
            total += it
        steps[extrap] = total
        if extrap:
            moves_x = moves
        else:
            assert moves == 0
    print(f"    steps extrapolated {steps[1]} ({moves_x} moves in the batches), plain {steps[0]}", flush=True)
    assert steps[1] <= steps[0]
    if kind == "grid":
        assert moves_x > 0 and steps[1] <= 0.7 * steps[0]


@pytest.mark.parametrize("tile", [512, 1024, 2048])
def test_merge_tile_sizes(tile):
    """CSR merge with 512 / 1024 / 2048 rows + entries per merge-path tile: a hub
    row longer than every tile, diff rows with more entries than the tile's LDS
    staging (read from memory instead), runs of empty rows; every batch merges."""
    n, s, d, w = hub_graph()
    say("merge tile", tile, "arcs", s.size)
    c = cfg(merge=-1.0)
    c.merge_tile = tile
    G = dg.Graph(n, s, d, w, config=c)
    q = G.sssp_attach(1)
    cs, cd, cw = s, d, w
    for i, (k, hub) in enumerate([(3000, 2500), (500, 0), (9000, 700)]):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 7300 + i)
        lo = 12500 + 800 * i
        extra_s = np.arange(lo, min(lo + hub, n), dtype=np.int32)
        bs = np.concatenate([bs, extra_s]); bd = np.concatenate([bd, np.zeros(extra_s.size, np.int32)])
        bw = np.concatenate([bw, np.full(extra_s.size, 5, np.int32)])
        bo = np.concatenate([bo, np.ones(extra_s.size, np.uint8)])
        st = G.apply(bs, bd, bw, bo)
        assert st.merged
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        assert_edges(G, cs, cd, cw)
        assert np.array_equal(q.read()[0], oracle.sssp(n, cs, cd, cw, 1))


@pytest.mark.parametrize("mode,pull,delta,sp", [(2, 0, 0, 0), (0, 0, 0, 0), (1, 0, 0, 0), (2, 1, 0, 0), (2, 0, 40, 0),
                                               (2, 0, 0, 2), (2, 0, 40, 2)])
def test_sssp_and_pagerank_together(mode, pull, delta, sp):
    """Two SSSP queries and PageRank on one graph: the SSSP updates run on a second
    stream beside the whole-graph tile steps (global form, pull 0), or after the
    steps where they cannot overlap (local form, per-vertex waves); host-driven
    steps (sp 0) or captured rounds replayed on the second stream (sp 2), plain
    or near-far (delta)."""
    n, s, d, w = hub_graph(seed=13)
    say("sssp + pagerank together, pr_mode", mode, "pull", pull, "delta", delta, "sssp schedule", sp)
    c = cfg(merge=0.02, delta=delta, persistent=sp)
    c.pr_mode = mode
    c.pr_pull = pull
    G = dg.Graph(n, s, d, w, config=c)
    qs = [G.sssp_attach(0), G.sssp_attach(5)]
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    cs, cd, cw = s, d, w
    for i, k in enumerate([3000, 40, 12000, 700]):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 7500 + i)
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        for q, src in zip(qs, (0, 5)):
            dist, par = q.read()
            assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, src)), (i, src)
        r, it, conv = qp.read()
        assert conv
        pr_check(r, n, cs, cd)


def test_undirected_all_queries_together():
    """SSSP, PageRank and triangles on one undirected graph: the SSSP update runs
    beside the PageRank steps, the triangle deltas before and after, merges
    included."""
    n, s, d = graphgen.rmat_undirected(11, 8 << 11, graphgen.config_seed(2, 77))[:3]
    w = graphgen.uniform_int(graphgen.config_seed(2, 78), 0, s.size, 1, 100).astype(np.int32)
    say("undirected sssp + pagerank + triangles")
    # Reading P7: on this graph (259 vertices of degree one) Jacobi stopped at an L1
    # step of 1e-9 can sit up to 1.4e-9 (max-abs) from the converged ranks, the oracle
    # run at 1e-9 included, so the ranks are pinned to the tight oracle (1e-14) and
    # the library's steps run to a hundredth of the tolerance.
    G = dg.Graph(n, s, d, w, undirected=True, config=cfg(merge=0.02, tol_scale=0.01))
    qs = G.sssp_attach(0)
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    qt = G.tc_attach()
    us, ud, uw = s, d, w
    merged = 0
    for i, k in enumerate([200, 1500, 30, 800]):
        bs, bd, bw, bo = graphgen.update_batch(n, us, ud, k, 8300 + i, undirected=True)
        merged += G.apply(bs, bd, bw, bo).merged
        us, ud, uw, _ = oracle.apply(n, us, ud, uw, bs, bd, bw, bo, undirected=True)
        both_s = np.concatenate([us, ud]); both_d = np.concatenate([ud, us]); both_w = np.concatenate([uw, uw])
        o = np.lexsort((both_d, both_s))
        cs, cd, cw = both_s[o], both_d[o], both_w[o]
        assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0)), i
        r, _, conv = qp.read()
        tight, _, _ = oracle.pagerank(n, cs, cd, 0.85, 1e-14, 5000)
        assert conv and abs(r.sum() - 1.0) < 1e-12
        assert float(np.max(np.abs(r - tight))) <= PR_MAXABS, i
        assert qt.read() == oracle.triangles(n, us, ud), i
    assert merged >= 1


@pytest.mark.parametrize("order,undirected", [(0, False), (1, False), (0, True)])
def test_vertex_order(order, undirected):
    """Vertex order inside the library (0: by degree, 1: as given): batches, SSSP
    distances and parents, PageRank, triangles and the exported edge list all come
    back in the caller's ids, equal to the oracle's.  The ids are shuffled first so
    that the degree order is far from the given one."""
    n, s, d, w = rmat_small(11, 12, 51)
    rng = np.random.default_rng(3)
    shuffle = rng.permutation(n).astype(np.int32)
    s, d = shuffle[s], shuffle[d]
    if undirected:
        key = np.unique((np.minimum(s, d).astype(np.int64) << 32) | np.maximum(s, d))
        s, d = (key >> 32).astype(np.int32), (key & 0xFFFFFFFF).astype(np.int32)
        w = np.ones(s.size, np.int32)
    else:
        o = np.lexsort((d, s))
        s, d, w = s[o], d[o], w[o]
    src = int(shuffle[0])
    say("vertex order", order, "undirected", undirected)
    c = cfg(merge=0.02)
    c.vertex_order = order
    G = dg.Graph(n, s, d, w if not undirected else None, undirected=undirected, config=c)
    if undirected:
        qt = G.tc_attach()
        assert qt.read() == oracle.triangles(n, s, d)
    else:
        qs = G.sssp_attach(src)
        qp = G.pr_attach(0.85, PR_TOL, 1000)
    cs, cd, cw = s, d, w
    for i, k in enumerate([300, 2000, 50, 900]):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, k, 8100 + i, undirected=undirected)
        G.apply(bs, bd, bw, bo)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo, undirected=undirected)
        assert_edges(G, cs, cd, cw, undirected=undirected)
        if undirected:
            assert qt.read() == oracle.triangles(n, cs, cd)
            continue
        dist, par = qs.read()
        assert np.array_equal(dist, oracle.sssp(n, cs, cd, cw, src)), i
        assert_tree(n, cs, cd, cw, src, dist, par)
        r, _, conv = qp.read()
        pr_check(r, n, cs, cd)
        sd, sp_ = G.sssp_static(src)
        assert np.array_equal(sd, dist)
        rs, _ = G.pr_static(0.85, PR_TOL, 1000)
        pr_check(rs, n, cs, cd)


@pytest.mark.parametrize("order", [0, 1])
def test_empty_graph_and_empty_batch(order):
    """An edgeless graph (every vertex dangling and isolated), an empty batch, a
    batch that inserts every edge, and one that deletes them all again."""
    n = 7
    e = np.zeros(0, np.int32)
    say("empty graph, vertex order", order)
    c = cfg()
    c.vertex_order = order
    G = dg.Graph(n, e, e, e, config=c)
    qs = G.sssp_attach(3)
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    dist, par = qs.read()
    assert dist.tolist() == [INF, INF, INF, 0, INF, INF, INF] and par.tolist() == [-1] * n
    r, _, _ = qp.read()
    assert np.allclose(r, 1.0 / n, atol=1e-15)
    st = G.apply(e, e, e, np.zeros(0, np.uint8))
    assert st.updates == 0
    s = np.array([3, 3, 0, 4, 6, 2], np.int32)
    d = np.array([0, 4, 1, 5, 3, 6], np.int32)
    w = np.array([5, 1, 2, 2, 7, 1], np.int32)
    G.apply(s, d, w, np.ones(6, np.uint8))
    cs, cd, cw, _ = oracle.apply(n, e, e, e, s, d, w, np.ones(6, np.uint8))
    assert_edges(G, cs, cd, cw)
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 3))
    pr_check(qp.read()[0], n, cs, cd)
    G.apply(s, d, w, np.zeros(6, np.uint8))
    assert G.info()["m"] == 0
    dist, par = qs.read()
    assert dist.tolist() == [INF, INF, INF, 0, INF, INF, INF] and par.tolist() == [-1] * n
    assert np.allclose(qp.read()[0], 1.0 / n, atol=1e-15)
    G.close()


def test_pagerank_dangling_and_isolated():
    say("pagerank dangling")
    # 0->1, 1 dangling, 2 isolated, 3->0, 3->1
    G = dg.Graph(4, [0, 3, 3], [1, 0, 1])
    q = G.pr_attach(0.85, 1e-12, 1000)
    r, _, _ = q.read()
    want, _, _ = oracle.pagerank(4, [0, 3, 3], [1, 0, 1], 0.85, 1e-14, 5000)
    assert np.max(np.abs(r - want)) < 1e-11
    G.apply([1, 3], [2, 0], [1, 0], [1, 0])  # 1->2 added, 3->0 deleted
    r, _, _ = q.read()
    want, _, _ = oracle.pagerank(4, [0, 3, 1], [1, 1, 2], 0.85, 1e-14, 5000)
    assert np.max(np.abs(r - want)) < 1e-11


def test_pagerank_local_form_many_dangling():
    """The local (listing) form stops on the L1 step of the normalised ranks, as
    the oracle does.  Half of the vertices lose every out-arc, so the unnormalised
    iterate sums to well below 1; the stopping rule must still match the oracle's
    at the same tolerance."""
    n, s, d, w = rmat_small(12, 16, 31)
    drop = graphgen.uniform01(77, 0, n) < 0.5
    keep = ~drop[s]
    s, d, w = s[keep], d[keep], w[keep]
    say("pagerank local form, many dangling vertices: n", n, "m", s.size, "dangling", int((np.bincount(s, minlength=n) == 0).sum()))
    c = cfg()
    c.pr_mode = 1
    G = dg.Graph(n, s, d, w, config=c)
    q = G.pr_attach(0.85, PR_TOL, 1000)
    cs, cd, cw = s, d, w
    for i, k in enumerate([40, 400, 4]):
        b = graphgen.update_batch(n, cs, cd, k, 8100 + i)
        st = G.apply(*b)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, *b)
        r, it, conv = q.read()
        want, _, oconv = oracle.pagerank(n, cs, cd, 0.85, PR_TOL, 1000)
        assert conv and oconv and st.pr_affected > 0
        assert float(np.max(np.abs(r - want))) <= PR_MAXABS, i
    G.close()


# ------------------------------------------------------------------ triangles

@pytest.mark.parametrize("heavy", [0, 16])
def test_tc_dynamic(heavy):
    n, u, v = graphgen.rmat_undirected(11, 16 << 11, 77)
    say("tc dynamic heavy", heavy)
    G = dg.Graph(n, u, v, None, undirected=True, config=cfg(heavy=heavy))
    q = G.tc_attach()
    assert q.read() == oracle.triangles(n, u, v)
    cu, cv = u, v
    for i, k in enumerate([10, 327, 3000, 1, 900]):
        bs, bd, bw, bo = graphgen.update_batch(n, cu, cv, k, 6000 + i, undirected=True)
        if i == 2:  # delete and re-insert some edges in the same batch
            bs = np.concatenate([bs, cu[:5], cv[:5]]).astype(np.int32)
            bd = np.concatenate([bd, cv[:5], cu[:5]]).astype(np.int32)
            bw = np.concatenate([bw, np.ones(10, np.int32)]).astype(np.int32)
            bo = np.concatenate([bo, np.zeros(5, np.uint8), np.ones(5, np.uint8)]).astype(np.uint8)
        G.apply(bs, bd, bw, bo)
        cu, cv, _, _ = oracle.apply(n, cu, cv, None, bs, bd, bw, bo, undirected=True)
        want = oracle.triangles(n, cu, cv)
        assert q.read() == want, i
        es, ed, _ = G.export()
        assert np.array_equal(es, cu) and np.array_equal(ed, cv)
    assert G.tc_static() == oracle.triangles(n, cu, cv)


def test_tc_two_hubs_split_rows():
    """Two hubs sharing 4,200 neighbours: the edge between them has a shorter row
    of about 5,200 entries, so its delta is cut into many work items and its
    longer row is searched through fences; batches mix it with edges of the same
    triangles (weights 6/2 and 6/3)."""
    say("tc two hubs, split rows")
    n, common = 7000, np.arange(2, 4202)
    only0, only1 = np.arange(4202, 5202), np.arange(5202, 6202)
    ring = np.arange(2, 6201)
    u = np.concatenate([[0], np.zeros(common.size + only0.size, np.int64), np.ones(common.size + only1.size, np.int64),
                        ring]).astype(np.int32)
    v = np.concatenate([[1], common, only0, common, only1, ring + 1]).astype(np.int32)
    G = dg.Graph(n, u, v, None, undirected=True)
    q = G.tc_attach()
    assert q.read() == oracle.triangles(n, u, v)
    cu, cv = u, v
    batches = [
        ([0], [1], [0]),                              # the hub edge alone: 4,200 triangles
        ([0, 0, 1, 2], [1, 2, 2, 3], [1, 0, 0, 0]),   # back in, with edges of its triangles out
        ([0, 0, 1, 5, 0], [1, 5, 5, 6, 2], [0, 1, 0, 0, 1]),
        ([1, 0, 9, 3000], [2, 1, 10, 3001], [1, 1, 0, 0]),
    ]
    for i, (bs, bd, bo) in enumerate(batches):
        bs, bd = np.array(bs, np.int32), np.array(bd, np.int32)
        bo, bw = np.array(bo, np.uint8), np.ones(len(bs), np.int32)
        G.apply(bs, bd, bw, bo)
        cu, cv, _, _ = oracle.apply(n, cu, cv, None, bs, bd, bw, bo, undirected=True)
        assert q.read() == oracle.triangles(n, cu, cv), i
    assert G.tc_static() == oracle.triangles(n, cu, cv)
    G.close()


def test_tc_small_closed_forms():
    say("tc closed forms")
    k = 9
    pairs = np.array([(a, b) for a in range(k) for b in range(a + 1, k)])
    G = dg.Graph(k, pairs[:, 0], pairs[:, 1], None, undirected=True)
    q = G.tc_attach()
    assert q.read() == 84
    # delete every edge of vertex 0: removes C(8,2) = 28 triangles
    G.apply(np.zeros(8, np.int32), np.arange(1, 9), None, np.zeros(8, np.uint8))
    assert q.read() == 84 - 28
    # insert them back: all triangles return
    G.apply(np.arange(1, 9), np.zeros(8, np.int32), None, np.ones(8, np.uint8))
    assert q.read() == 84


# ------------------------------------------------------------------ snapshots, batches, device memory

def test_snapshot_restore_repeats_a_batch():
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("snapshot")
    G = dg.Graph(n, s, d, w)
    qs, qp = G.sssp_attach(0), G.pr_attach()
    G.snapshot()
    G.apply(bs, bd, bw, bo)
    d1, r1 = qs.read()[0], qp.read()[0]
    e1 = G.export()
    G.restore()
    assert np.array_equal(G.export()[0], s[np.lexsort((d, s))])
    G.apply(bs, bd, bw, bo)
    assert np.array_equal(qs.read()[0], d1)
    assert np.array_equal(qp.read()[0], r1)  # deterministic reductions
    for x, y in zip(G.export(), e1):
        assert np.array_equal(x, y)


def test_batch_size_chunks_match_one_shot():
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("batch_size chunks")
    G1 = dg.Graph(n, s, d, w)
    G2 = dg.Graph(n, s, d, w)
    q1, q2 = G1.sssp_attach(0), G2.sssp_attach(0)
    G1.apply(bs, bd, bw, bo)
    st = G2.apply(bs, bd, bw, bo, batch_size=500)
    assert st.chunks == (bs.size + 499) // 500
    # chunked application is sequential application of the chunks
    cs, cd, cw = s, d, w
    for o in range(0, bs.size, 500):
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs[o:o + 500], bd[o:o + 500], bw[o:o + 500], bo[o:o + 500])
    assert_edges(G2, cs, cd, cw)
    assert np.array_equal(q2.read()[0], oracle.sssp(n, cs, cd, cw, 0))


def test_device_pointer_batch():
    import torch
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("device pointers")
    dev = torch.device("cuda:0")
    G = dg.Graph(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev), torch.from_numpy(w).to(dev))
    q = G.sssp_attach(0)
    G.set_stream(torch.cuda.current_stream().cuda_stream)
    G.apply(torch.from_numpy(bs).to(dev), torch.from_numpy(bd).to(dev), torch.from_numpy(bw).to(dev),
            torch.from_numpy(bo).to(dev))
    out = torch.empty(n, dtype=torch.int32, device=dev)
    q.read(out)
    torch.cuda.synchronize()
    cs, cd, cw, _ = oracle.apply(n, s, d, w, bs, bd, bw, bo)
    assert np.array_equal(out.cpu().numpy(), oracle.sssp(n, cs, cd, cw, 0))


def test_partially_dynamic_modes():
    """Incremental-only and decremental-only batches (no op array) against the
    oracle; an op that contradicts the mode rejects the batch before any change."""
    n, s, d, w = rmat_small(11, 8, 41)
    say("incremental / decremental modes")
    G = dg.Graph(n, s, d, w)
    qs, qp = G.sssp_attach(0), G.pr_attach(0.85, PR_TOL, 1000)
    b = graphgen.update_batch(n, s, d, 600, 4100)
    ins = b[3] == 1
    G.insert(b[0][ins], b[1][ins], b[2][ins])
    cs, cd, cw, ost = oracle.apply(n, s, d, w, b[0][ins], b[1][ins], b[2][ins], b[3][ins])
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0))
    pr_check(qp.read()[0], n, cs, cd)
    G.delete(cs[:300], cd[:300])
    cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, cs[:300], cd[:300], np.zeros(300, np.int32),
                                 np.zeros(300, np.uint8))
    assert_edges(G, cs, cd, cw)
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0))
    pr_check(qp.read()[0], n, cs, cd)
    before = G.export()
    with pytest.raises(dg.DGError) as e:  # an insertion in a decremental batch
        G.apply(cs[:4], cd[:4], cw[:4], np.array([0, 0, 1, 0], np.uint8), mode=dg.DG_DECREMENTAL)
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError) as e:
        G.apply(cs[:4], cd[:4], cw[:4], None, mode=dg.DG_DECREMENTAL | dg.DG_INCREMENTAL)
    assert e.value.code == dg.DG_EINVAL
    for x, y in zip(before, G.export()):
        assert np.array_equal(x, y)


def test_merge_period():
    """merge_period = 3 with the size threshold off: every third batch merges."""
    n, s, d, w = rmat_small(10, 8, 43)
    say("merge period")
    c = cfg(merge=1e9)
    c.merge_period = 3
    G = dg.Graph(n, s, d, w, config=c)
    q = G.sssp_attach(0)
    cs, cd, cw = s, d, w
    merged = []
    for i in range(7):
        bs, bd, bw, bo = graphgen.update_batch(n, cs, cd, 80, 4200 + i)
        merged.append(G.apply(bs, bd, bw, bo).merged)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, bs, bd, bw, bo)
        assert_edges(G, cs, cd, cw)
        assert np.array_equal(q.read()[0], oracle.sssp(n, cs, cd, cw, 0))
    assert merged == [0, 0, 1, 0, 0, 1, 0]

# ------------------------------------------------------------------ residual push (pr_mode 3)

def pr_cfg(mode, **kw):
    c = cfg(**kw)
    c.pr_mode = mode
    return c


@pytest.mark.parametrize("kind", ["rmat", "grid", "undirected"])
def test_pagerank_residual_push_matches_oracle(kind):
    """Residual push after each batch: ranks within max-abs 1e-10 of the oracle's
    power iteration, converged, on a directed R-MAT with dangling vertices, a grid
    (batches with long-range inserts) and an undirected graph, with SSSP attached
    on the directed ones (it runs after the push)."""
    say("pagerank residual push", kind)
    und = kind == "undirected"
    if kind == "rmat":
        n, s, d, w = rmat_small(12, 8, 81)
        sizes = [400, 40, 4, 1200]
    elif kind == "grid":
        n, s, d, w = graphgen.c2g_graph(96)
        sizes = [60, 6, 600, 1]
    else:
        n, s, d = graphgen.rmat_undirected(11, 8 << 11, graphgen.config_seed(2, 81))
        w = None
        sizes = [300, 30, 3]
    # the undirected R-MAT has hundreds of degree-one vertices: the reading of the
    # tolerance pair that its all-queries test follows applies (steps at a
    # hundredth of the tolerance, ranks pinned to the tight oracle)
    G = dg.Graph(n, s, d, w, undirected=und, config=pr_cfg(3, tol_scale=0.01 if und else 0.0))
    otol = 1e-14 if und else PR_TOL
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    qs = None if und else G.sssp_attach(0)
    cs, cd, cw = s, d, (w if w is not None else np.ones(s.size, np.int32))

    def arcs(a, b):  # an undirected edge is an arc each way for PageRank
        return (np.concatenate([a, b]), np.concatenate([b, a])) if und else (a, b)

    rank, _, conv = qp.read()
    want, _, _ = oracle.pagerank(n, *arcs(cs, cd), 0.85, otol, 1000)
    assert conv and float(np.max(np.abs(rank - want))) <= PR_MAXABS
    for i, k in enumerate(sizes):
        b = graphgen.update_batch(n, cs, cd, k, graphgen.config_seed(0, 810 + i), wmax=1000 if kind == "grid" else 100,
                                  undirected=und)
        st = G.apply(*b)
        cs, cd, cw, _ = oracle.apply(n, cs, cd, cw, *b, undirected=und)
        rank, it, conv = qp.read()
        want, _, oconv = oracle.pagerank(n, *arcs(cs, cd), 0.85, otol, 1000)
        err = float(np.max(np.abs(rank - want)))
        say("  batch", i, "k", k, "rounds", it, "pushed arcs", st.edges_traversed, "max-abs", err)
        assert conv and oconv and err <= PR_MAXABS
        assert abs(float(rank.sum()) - 1.0) <= 1e-12
        if qs is not None:
            assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0))
    G.close()


def test_pagerank_residual_push_stays_local_on_grid():
    """On a grid (no dangling mass, long paths) a small batch's push examines far
    fewer arcs than the sweeps of the global form, which pull every arc per step;
    both land within the tolerance of the oracle."""
    n, s, d, w = graphgen.c2g_graph(128)
    b = graphgen.update_batch(n, s, d, 4, graphgen.config_seed(0, 820), wmax=1000)
    cs, cd, cw, _ = oracle.apply(n, s, d, w, *b)
    want, _, _ = oracle.pagerank(n, cs, cd, 0.85, PR_TOL, 1000)
    say("residual push locality on a 128^2 grid, 4 updates")
    arcs = {}
    for mode in (2, 3):
        G = dg.Graph(n, s, d, w, config=pr_cfg(mode))
        qp = G.pr_attach(0.85, PR_TOL, 1000)
        st = G.apply(*b)
        rank, _, conv = qp.read()
        assert conv and float(np.max(np.abs(rank - want))) <= PR_MAXABS
        arcs[mode] = st.edges_traversed
        G.close()
    say("  arcs examined: global sweeps", arcs[2], "push", arcs[3])
    assert 0 < arcs[3] < arcs[2] / 3


def test_pagerank_residual_push_snapshot_restore():
    n, s, d, w = rmat_small(11, 8, 83)
    b1 = graphgen.update_batch(n, s, d, 300, graphgen.config_seed(0, 830))
    say("residual push snapshot/restore")
    G = dg.Graph(n, s, d, w, config=pr_cfg(3))
    qp = G.pr_attach(0.85, PR_TOL, 1000)
    G.snapshot()
    G.apply(*b1)
    r1, _, _ = qp.read()
    G.restore()
    G.apply(*b1)
    r2, _, _ = qp.read()
    cs, cd, _, _ = oracle.apply(n, s, d, w, *b1)
    want, _, _ = oracle.pagerank(n, cs, cd, 0.85, PR_TOL, 1000)
    assert float(np.max(np.abs(r1 - want))) <= PR_MAXABS and float(np.max(np.abs(r2 - want))) <= PR_MAXABS
    assert float(np.max(np.abs(r1 - r2))) <= 1e-13  # atomics reorder sums: equal up to rounding
    G.close()


def test_tc_random_sequences_match_recount():
    """Random batch sequences on small undirected graphs (merge thresholds 0.05,
    every batch, never and 0.2; slot reuse on and off; every third batch followed
    by its exact inverse): after every batch the maintained count equals the
    static forward recount, and after each sequence the oracle's count."""
    rng = np.random.default_rng(17)
    for trial in range(16):
        sc = int(rng.integers(7, 12))
        n, u, v = graphgen.rmat_undirected(sc, int(rng.integers(4, 16)) << sc, int(rng.integers(1, 1 << 30)))
        c = cfg(merge=float(rng.choice([0.05, -1.0, 1e9, 0.2])))
        c.diff_only = int(rng.integers(0, 2))
        say("tc random sequence", trial, "scale", sc, "merge", c.merge_threshold, "diff_only", c.diff_only)
        G = dg.Graph(n, u, v, None, undirected=True, config=c)
        q = G.tc_attach()
        cu, cv = u, v
        for i in range(10):
            k = int(np.exp(rng.uniform(np.log(4), np.log(min(2000, max(8, cu.size))))))
            b = graphgen.update_batch(n, cu, cv, k, int(rng.integers(1, 1 << 30)), undirected=True)
            inv = (b[0].copy(), b[1].copy(), np.ones(b[0].size, np.int32), (b[3] == 0).astype(np.uint8))
            for bb in ((b, inv) if i % 3 == 0 else (b,)):
                G.apply(*bb)
                cu, cv, _, _ = oracle.apply(n, cu, cv, None, *bb, undirected=True)
                assert q.read() == G.tc_static(), (trial, i)
        assert q.read() == oracle.triangles(n, cu, cv), trial
        G.close()



def test_pr_gather_floor():
    """dg_pr_gather_floor: a positive time on a graph with edges, zero on an
    edgeless one, and a refusal of reps < 1."""
    n, s, d, w = rmat_small(scale=12)
    say("gather floor")
    G = dg.Graph(n, s, d, w)
    assert G.pr_gather_floor(3) > 0.0
    with pytest.raises(dg.DGError):
        G.pr_gather_floor(0)
    e = np.zeros(0, np.int32)
    E = dg.Graph(5, e, e, e)
    assert E.pr_gather_floor(1) == 0.0


def test_calibration_kernels():
    """dg_calibrate: every kind runs on a device buffer; the stream read keeps the
    buffer, the stream write fills it; kinds outside 0..3, sizes that are not a
    multiple of 4 KiB and kind 3 below 64 KiB are refused."""
    import ctypes
    import torch

    say("calibration kernels")
    lib = dg.load_library()
    buf = torch.full((1 << 20,), 7, dtype=torch.uint8, device="cuda:0")
    ptr = ctypes.c_void_p(buf.data_ptr())
    dg._check(lib.dg_calibrate(0, ptr, buf.numel(), None))
    assert int(buf[(1 << 19):].min()) == 7 and int(buf[(1 << 19):].max()) == 7
    for kind in (1, 2, 3):
        dg._check(lib.dg_calibrate(kind, ptr, buf.numel(), None))
    torch.cuda.synchronize()
    for kind, size in ((4, buf.numel()), (0, 5000), (3, 32 << 10)):
        with pytest.raises(dg.DGError):
            dg._check(lib.dg_calibrate(kind, ptr, size, None))


@pytest.mark.parametrize("persistent", [0, 2])
def test_traversal_tally(persistent):
    """edges_traversed counts the entries the update examined: positive for an
    SSSP-only batch (host-driven steps or captured rounds) and for a triangle
    batch, and no more than every arc once per step."""
    n, s, d, w = rmat_small(11, 8, 41)
    say("traversal tally, sssp schedule", persistent)
    G = dg.Graph(n, s, d, w, config=cfg(persistent=persistent))
    G.sssp_attach(0)
    bs, bd, bw, bo = graphgen.update_batch(n, s, d, 400, 4100)
    st = G.apply(bs, bd, bw, bo)
    assert st.sssp_steps > 0
    assert 0 < st.edges_traversed <= (st.sssp_steps + 20) * (s.size + 400)
    un, us, ud = graphgen.rmat_undirected(10, 4000, 42)
    T = dg.Graph(un, us, ud, None, undirected=True)
    T.tc_attach()
    bs, bd, bw, bo = graphgen.update_batch(un, us, ud, 300, 4101, undirected=True)
    st = T.apply(bs, bd, bw, bo)
    assert st.edges_traversed > 0
