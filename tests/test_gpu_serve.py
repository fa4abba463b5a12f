"""Serving loop: every answer equals the oracle on the evolving graph, and equals
the answer of the same request sequence run alone (one worker, one request at a
time) when requests of many graphs run mixed on several workers."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def make_graphs(count, seed):
    gs = []
    for i in range(count):
        sc = 8 + (i % 4)
        gs.append(graphgen.rmat_directed(sc, 8 << sc, seed * 100 + i))
    return gs


def make_requests(graphs, count, seed, kmin=4, kmax=400, tc_max_n=None):
    """Request stream: graph uniform, batch log-uniform in [kmin, kmax], kinds
    40/40/20 (a triangle request on a graph above tc_max_n vertices becomes a
    PageRank request, to keep the oracle's recount short)."""
    rng_g = graphgen.uniform_int(graphgen.stream_seed(seed, "misc"), 0, count, 0, len(graphs) - 1)
    rng_k = graphgen.uniform01(graphgen.stream_seed(seed, "w"), 0, count)
    rng_q = graphgen.uniform01(graphgen.stream_seed(seed, "perm"), 0, count)
    cur = [(n, s, d, w) for n, s, d, w in graphs]
    reqs = []
    for i in range(count):
        gi = int(rng_g[i])
        n, s, d, w = cur[gi]
        k = int(round(np.exp(np.log(kmin) + rng_k[i] * (np.log(kmax) - np.log(kmin)))))
        k = min(k, 2 * s.size)
        b = graphgen.update_batch(n, s, d, k, seed * 1000 + i)
        kind = dg.SSSP if rng_q[i] < 0.4 else (dg.PAGERANK if rng_q[i] < 0.8 else dg.TRIANGLES)
        if kind == dg.TRIANGLES and tc_max_n is not None and n > tc_max_n:
            kind = dg.PAGERANK
        source = int((seed * 31 + i * 17) % n)
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *b)
        cur[gi] = (n, s2, d2, w2)
        reqs.append((gi, kind, source, b, (n, s2, d2, w2)))
    return reqs


def run(graphs, reqs, workers, all_at_once):
    S = dg.Server(workers=workers)
    for n, s, d, w in graphs:
        S.add_graph(n, s, d, w)
    S.start()
    out = []
    if all_at_once:
        tickets = [S.submit(gi, kind, *b, source=src) for gi, kind, src, b, _ in reqs]
        for t in tickets:
            out.append(S.wait(t))
    else:
        for gi, kind, src, b, _ in reqs:
            out.append(S.wait(S.submit(gi, kind, *b, source=src)))
    S.close()
    return out


def check_answers(reqs, alone, mix):
    for i, ((gi, kind, src, b, (n, s2, d2, w2)), (ra, oa), (rm, om)) in enumerate(zip(reqs, alone, mix)):
        assert ra.status == 0 and rm.status == 0, i
        if kind == dg.SSSP:
            want = oracle.sssp(n, s2, d2, w2, src)
            assert np.array_equal(oa, want) and np.array_equal(om, want), i
        elif kind == dg.PAGERANK:
            want, _, _ = oracle.pagerank(n, s2, d2, 0.85, 1e-9, 1000)
            assert np.max(np.abs(oa - want)) <= 1e-10, i
            assert np.array_equal(oa, om), i  # deterministic reductions: bit-equal alone and mixed
        else:
            u, v = oracle.symmetrise(s2, d2)
            want = oracle.triangles(n, u, v)
            assert ra.tc == want and rm.tc == want, i
        assert ra.t_submit <= ra.t_start <= ra.t_end


def test_serve_mix_equals_alone_and_oracle():
    graphs = make_graphs(6, 3)
    reqs = make_requests(graphs, 40, 5)
    say("serve alone")
    alone = run(graphs, reqs, workers=1, all_at_once=False)
    say("serve mix")
    mix = run(graphs, reqs, workers=4, all_at_once=True)
    check_answers(reqs, alone, mix)


def test_serve_config_sizes_sample():
    """The serving workload's shapes on a sample of its graphs: R-MAT scales 12,
    15, 17 and 20 with 16 arcs per vertex, batches log-uniform in [100, 10^5],
    query kinds 40/40/20 (triangles on the graphs up to scale 17)."""
    graphs = [graphgen.rmat_directed(sc, 16 << sc, graphgen.config_seed(4, 50 + sc)) for sc in (12, 15, 17, 20)]
    reqs = make_requests(graphs, 14, 6, kmin=100, kmax=100000, tc_max_n=1 << 17)
    say("serve at the workload's sizes: batches", [len(r[3][0]) for r in reqs], "kinds", [r[1] for r in reqs])
    alone = run(graphs, reqs, workers=1, all_at_once=False)
    say("serve at the workload's sizes, mixed")
    mix = run(graphs, reqs, workers=4, all_at_once=True)
    say("oracle answers")
    check_answers(reqs, alone, mix)


def test_serve_admission_errors():
    graphs = make_graphs(2, 4)
    say("serve admission")
    S = dg.Server(workers=1, budget_bytes=1 << 21, max_waiting=1)
    for n, s, d, w in graphs:
        S.add_graph(n, s, d, w)
    n, s, d, w = graphs[0]
    # 20,000 insertions (duplicates allowed: the request is refused before it runs)
    big = (graphgen.uniform_int(9, 0, 20000, 0, n - 1).astype(np.int32),
           graphgen.uniform_int(10, 0, 20000, 0, n - 1).astype(np.int32),
           np.ones(20000, np.int32), np.ones(20000, np.uint8))
    with pytest.raises(dg.DGError) as e:
        S.submit(0, dg.TRIANGLES, *big)
    assert e.value.code == dg.DG_EBUDGET
    # before start nothing runs: the second waiting request exceeds max_waiting
    small = graphgen.update_batch(n, s, d, 4, 10)
    t = S.submit(0, dg.TRIANGLES, *small)
    with pytest.raises(dg.DGError) as e:
        S.submit(1, dg.TRIANGLES, *small)
    assert e.value.code == dg.DG_EBUSY
    S.start()
    res, _ = S.wait(t)
    assert res.status == 0
    S.close()
