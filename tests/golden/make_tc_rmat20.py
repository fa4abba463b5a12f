"""Writes tc_rmat20.json: exact triangle counts of the undirected R-MAT scale-20
workload (16 * 2^20 edges) before and after three update batches of 0.1 %, 1 %
and 5 % of its edges, applied in that order.

Every value comes from the oracle (edge-list application, then the node-iterator
count); the inputs come from graphgen with the seeds recorded in the file.  Run
from the repository root:

    python tests/golden/make_tc_rmat20.py

It takes several minutes: the four counts run in parallel processes.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

SCALE = 20
PCTS = (0.001, 0.01, 0.05)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tc_rmat20.json")


def batch_seed(i: int) -> int:
    return graphgen.config_seed(2, 200 + i)


def workload():
    """The graph and its three batches, each drawn against the initial graph."""
    n, s, d = graphgen.c3_graph(SCALE)[:3]
    keys = graphgen.edge_keys(s, d, True)
    bats = [graphgen.update_batch(n, s, d, int(p * s.size), batch_seed(i), undirected=True, existing=keys)
            for i, p in enumerate(PCTS)]
    return n, s, d, bats


def _count(args):
    n, u, v = args
    t0 = time.perf_counter()
    c = oracle.triangles(n, u, v)
    return c, time.perf_counter() - t0


def main() -> None:
    n, s, d, bats = workload()
    graphs = [(s, d)]
    stats = []
    cs, cd = s, d
    for b in bats:
        cs, cd, _, st = oracle.apply(n, cs, cd, np.ones(cs.size, np.int32), *b, undirected=True)
        graphs.append((cs, cd))
        stats.append(st)
    with ProcessPoolExecutor(max_workers=len(graphs)) as ex:
        res = list(ex.map(_count, [(n, u, v) for u, v in graphs]))
    doc = {
        "what": "triangle counts of the undirected R-MAT scale-20 workload after each batch (oracle)",
        "graph": {"generator": "graphgen.c3_graph", "scale": SCALE, "vertices": int(n), "edges": int(s.size)},
        "batches": [{"pct": p, "k": int(len(b[0])), "seed": batch_seed(i),
                     "deleted": st[0], "inserted": st[1], "ignored_del": st[2], "ignored_ins": st[3]}
                    for i, (p, b, st) in enumerate(zip(PCTS, bats, stats))],
        "counts": [int(c) for c, _ in res],
        "oracle_seconds": [round(t, 1) for _, t in res],
        "command": "python tests/golden/make_tc_rmat20.py",
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps(doc, indent=1))


if __name__ == "__main__":
    main()
