"""GPU parity of batched sets of graphs (one store, one captured update per batch)
and of the autotuner, against the CPU oracle."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def members(count, seed, smin=5, smax=10, deg=8):
    out = []
    scales = graphgen.uniform_int(graphgen.stream_seed(seed, "misc"), 0, count, smin, smax)
    for i, sc in enumerate(scales.tolist()):
        n, s, d, w = graphgen.rmat_directed(sc, deg << sc, seed * 1000 + i)
        out.append((n, s, d, w))
    return out


def member_batches(mem, seed, lo=0.01, hi=0.10):
    fr = graphgen.uniform01(graphgen.stream_seed(seed, "misc"), 7, len(mem)) * (hi - lo) + lo
    out = []
    for i, ((n, s, d, w), f) in enumerate(zip(mem, fr.tolist())):
        k = max(2, int(f * s.size))
        out.append(graphgen.update_batch(n, s, d, k, seed * 7919 + i))
    return out


@pytest.mark.parametrize("mode", [2, 1])
def test_set_matches_oracle_over_batches(mode):
    """mode 2: captured frontier rounds (default); mode 1: persistent work queue."""
    mem = members(24, 11)
    say("set of", len(mem), "mode", mode)
    c = dg.Config()
    c.sssp_persistent = mode
    S = dg.GraphSet(mem, config=c)
    info = S.info()
    assert info["count"] == 24 and info["vertices"] == sum(m[0] for m in mem)
    S.sssp_attach(np.zeros(len(mem), np.int32))
    for i, (n, s, d, w) in enumerate(mem):
        assert np.array_equal(S.read(i)[0], oracle.sssp(n, s, d, w, 0)), i
    cur = list(mem)
    for rnd in range(4):
        bats = member_batches(cur, 100 + rnd)
        st = S.apply(bats)
        assert st.updates == sum(len(b[0]) for b in bats)
        nxt = []
        for i, ((n, s, d, w), b) in enumerate(zip(cur, bats)):
            s2, d2, w2, _ = oracle.apply(n, s, d, w, *b)
            nxt.append((n, s2, d2, w2))
            dist, par = S.read(i)
            assert np.array_equal(dist, oracle.sssp(n, s2, d2, w2, 0)), (rnd, i)
            if i % 8 == 0:  # parents form a shortest-path tree in member-local ids
                emap = {(a, b_): c for a, b_, c in zip(s2.tolist(), d2.tolist(), w2.tolist())}
                for v in range(n):
                    if v and dist[v] < dg.DG_INF:
                        assert dist[par[v]] + emap[(int(par[v]), v)] == dist[v]
        cur = nxt
    gs = S.graph_stats()
    # one replay per batch (queue) or two (cut walk, push rounds); layouts alternate
    assert gs["launches"] == 4 * (2 if mode == 2 else 1) and 1 <= gs["captures"] <= gs["launches"]


@pytest.mark.parametrize("mode", [2, 1])
def test_set_members_with_empty_batches(mode):
    """Members with no updates: a leading one, a trailing one and a run of ten in
    the middle, with enough updates in total that the 256-entry translation blocks
    begin inside and next to the empty members."""
    mem = members(40, 17, 6, 9)
    bats = member_batches(mem, 300)
    empty = [0, *range(12, 22), 39]
    e = (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8))
    for i in empty:
        bats[i] = e
    total = sum(len(b[0]) for b in bats)
    say("set with empty member batches, mode", mode, "updates", total)
    assert total > 4 * 256
    c = dg.Config()
    c.sssp_persistent = mode
    S = dg.GraphSet(mem, config=c)
    S.sssp_attach(np.zeros(len(mem), np.int32))
    st = S.apply(bats)
    assert st.updates == total
    for i, (n, s, d, w) in enumerate(mem):
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *bats[i])
        assert np.array_equal(S.read(i)[0], oracle.sssp(n, s2, d2, w2, 0)), i
    S.close()


def test_set_member_equals_alone():
    mem = members(6, 12, 8, 10)
    say("set vs alone")
    S = dg.GraphSet(mem)
    S.sssp_attach(np.full(len(mem), 3, np.int32))
    bats = member_batches(mem, 200)
    S.apply(bats)
    for i, (n, s, d, w) in enumerate(mem):
        G = dg.Graph(n, s, d, w)
        q = G.sssp_attach(3)
        G.apply(*bats[i])
        assert np.array_equal(S.read(i)[0], q.read()[0])


def test_set_rejects_out_of_member_ids():
    mem = members(4, 13, 5, 6)
    say("set bad ids")
    S = dg.GraphSet(mem)
    S.sssp_attach(np.zeros(4, np.int32))
    before = [S.read(i)[0].copy() for i in range(4)]
    bats = member_batches(mem, 300)
    n0 = mem[0][0]
    bad = list(bats)
    bad[0] = (np.array([0], np.int32), np.array([n0], np.int32), np.array([1], np.int32), np.array([1], np.uint8))
    with pytest.raises(dg.DGError) as e:
        S.apply(bad)
    assert e.value.code == dg.DG_EINVAL
    for i in range(4):
        assert np.array_equal(S.read(i)[0], before[i])


def test_set_autotune_keeps_state():
    mem = members(10, 14, 6, 9)
    say("set autotune")
    S = dg.GraphSet(mem)
    S.sssp_attach(np.zeros(len(mem), np.int32))
    bats = member_batches(mem, 400)
    best, ms = S.autotune(bats)
    assert best.heavy_degree in (32, 64, 128, 256, 512) and ms > 0
    for i, (n, s, d, w) in enumerate(mem):  # tuning rolled every trial back
        assert np.array_equal(S.read(i)[0], oracle.sssp(n, s, d, w, 0))
    S.apply(bats)
    for i, ((n, s, d, w), b) in enumerate(zip(mem, bats)):
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *b)
        assert np.array_equal(S.read(i)[0], oracle.sssp(n, s2, d2, w2, 0))


def test_graph_autotune_keeps_state():
    n, s, d, w, (bs, bd, bw, bo) = graphgen.c1_workload()
    say("graph autotune")
    G = dg.Graph(n, s, d, w)
    qs, qp = G.sssp_attach(0), G.pr_attach()
    before = G.export()
    best, ms = dg.autotune(G, bs, bd, bw, bo)
    assert best.heavy_degree in (32, 64, 128, 256, 512)
    for x, y in zip(G.export(), before):
        assert np.array_equal(x, y)
    assert np.array_equal(qs.read()[0], oracle.sssp(n, s, d, w, 0))
    G.apply(bs, bd, bw, bo)
    cs, cd, cw, _ = oracle.apply(n, s, d, w, bs, bd, bw, bo)
    assert np.array_equal(qs.read()[0], oracle.sssp(n, cs, cd, cw, 0))
