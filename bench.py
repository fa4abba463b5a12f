#!/usr/bin/env python3
"""Dynamic-graph update throughput on one MI355X.

Workload (one step): a batch of updates (default 100,000: half deletions of
existing arcs, half insertions of new uniform arcs, weights U[1,100]) applied to
a directed R-MAT scale-22 graph (4,194,304 vertices, 67,108,864 arcs, a=0.57
b=0.19 c=0.19, weights U[1,100]) that keeps a shortest-path query from vertex 0
and a PageRank query (damping 0.85, L1 tolerance 1e-9, FP64) current.  Every
step gets its own batch (all drawn against the initial graph); the batches are
resident in HBM before the timed region.  value = updates applied per second of
wall time over the timed steps.

Also reported: the static-recompute GPU path on the same graph (batch apply
plus SSSP and PageRank from scratch), the roofline of the dominant kernel (the
PageRank pull) from HIP-event launch timing inside this run, and the CPU oracle
(edge-list apply + Dijkstra + FP64 power iteration) timed on the host for one
batch.  One GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "dyn SSSP/PR/TC updates/sec + HBM GB/s vs static recompute; serve p50/p99"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--batch", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-static", action="store_true")
    ap.add_argument("--heavy-degree", type=int, default=0, help="rows longer than this are split (0: library default)")
    ap.add_argument("--sssp-persistent", type=int, default=0, help="1: SSSP on the single-launch work queue")
    ap.add_argument("--pr-mode", type=int, default=0, help="PageRank form after a batch: 0 auto, 1 local, 2 global")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run five plain 256 MiB device-to-device copies (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": int(a.numel()), "copies": 5}), flush=True)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the dynamic-graph hot path on one GPU; this build runs on a single "
              "MI355X, so --gpus must be 1 (multi-GPU sharding is a design note, not a measured path).",
              file=sys.stderr)
        return 2

    import torch

    import graphgen
    import paper_2507_11094_amd as dg

    dev = torch.device("cuda:0")
    K, W, k = args.steps, args.warmup, args.batch
    t = time.perf_counter()
    n, s, d, w = graphgen.rmat_directed(args.scale, 16 << args.scale, graphgen.config_seed(1, 0))
    log(f"graph n={n} m={s.size} generated in {time.perf_counter() - t:.1f}s")
    keys = graphgen.edge_keys(s, d)
    batches = []
    for i in range(W + K):
        batches.append(graphgen.update_batch(n, s, d, k, graphgen.config_seed(1, 100 + i), existing=keys))
    log(f"{W + K} batches of {k} drawn")
    dbatches = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in b) for b in batches]
    torch.cuda.synchronize()

    t = time.perf_counter()
    cfg = dg.Config()
    cfg.heavy_degree = args.heavy_degree
    cfg.sssp_persistent = args.sssp_persistent
    cfg.pr_mode = args.pr_mode
    G = dg.Graph(n, s, d, w, config=cfg)
    log(f"graph built on device in {time.perf_counter() - t:.2f}s")
    t = time.perf_counter()
    qs = G.sssp_attach(0)
    qp = G.pr_attach(0.85, 1e-9, 1000)
    log(f"queries attached (static solves) in {time.perf_counter() - t:.2f}s")

    for i in range(W):
        G.apply(*dbatches[i])
        log(f"warmup {i + 1}/{W}")
    dg.dg_profile_enable(True)
    dg.dg_profile_reset()
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        st = G.apply(*dbatches[W + i])
        stats.append(st.as_dict())
        log(f"step {i + 1}/{K}: {st.t_total_ms:.2f} ms (sssp {st.t_sssp_ms:.2f}, pr {st.t_pr_ms:.2f}, "
            f"update {st.t_update_ms + st.t_validate_ms:.2f}, merge {st.t_merge_ms:.2f}, "
            f"pr_iters {st.pr_iterations}, |A| {st.pr_affected})")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = dg.dg_profile_read()
    dg.dg_profile_enable(False)
    elapsed = t1 - t0
    value = K * k / elapsed
    ms_per_step = 1e3 * elapsed / K

    def avg(key):
        return float(np.mean([x[key] for x in stats]))

    pull = prof.get("pr_pull", {"launches": 0, "ms": 0.0, "bytes": 0.0})
    achieved = pull["bytes"] / (pull["ms"] * 1e-3) / 1e9 if pull["ms"] > 0 else 0.0
    roofline = {
        "kernel": "k_pr_pull",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "launches": pull["launches"],
        "avg_launch_us": round(1e3 * pull["ms"] / max(pull["launches"], 1), 2),
        "alg_bytes_per_launch": round(pull["bytes"] / max(pull["launches"], 1)),
    }
    kernels = {name: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2),
                      "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
               for name, v in prof.items()}

    static = None
    if not args.no_static:
        torch.cuda.synchronize()
        t = time.perf_counter()
        G.sssp_static(0)
        t_ss = time.perf_counter() - t
        t = time.perf_counter()
        _, it_pr = G.pr_static(0.85, 1e-9, 1000)
        t_ps = time.perf_counter() - t
        t_apply = 1e-3 * (avg("t_validate_ms") + avg("t_update_ms") + avg("t_merge_ms"))
        static = {
            "sssp_ms": round(1e3 * t_ss, 3),
            "pr_ms": round(1e3 * t_ps, 3),
            "pr_iterations": it_pr,
            "apply_ms": round(1e3 * t_apply, 3),
            "updates_per_s": round(k / (t_apply + t_ss + t_ps), 1),
            "dynamic_speedup": round((t_apply + t_ss + t_ps) / (elapsed / K), 3),
        }
        log(f"static recompute: sssp {1e3 * t_ss:.1f} ms, pr {1e3 * t_ps:.1f} ms ({it_pr} iters)")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        log("cpu oracle on one batch (apply + Dijkstra + power iteration) ...")
        b = batches[W]
        t = time.perf_counter()
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *b)
        oracle.sssp(n, s2, d2, w2, 0)
        oracle.pagerank(n, s2, d2, 0.85, 1e-9, 1000)
        t_cpu = time.perf_counter() - t
        cpu = {"value": round(k / t_cpu, 1), "unit": "updates/s", "cores": 1, "kind": "oracle",
               "seconds": round(t_cpu, 2),
               "sample": f"one {k}-update batch on the full R-MAT scale-{args.scale} graph: edge-list "
                         f"apply, Dijkstra from 0, FP64 power iteration to L1 1e-9 (single thread)"}
        log(f"cpu oracle: {t_cpu:.1f}s")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f64",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}-dynamic-sssp+pagerank", "vertices": n, "arcs": int(s.size),
                   "batch": k, "insert_fraction": 0.5, "queries": ["sssp(0)", "pagerank(0.85, l1 1e-9)"],
                   "parallelism": "1 gpu", "heavy_degree": args.heavy_degree or 512,
                   "sssp_persistent": args.sssp_persistent, "pr_mode": args.pr_mode},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "static_recompute": static,
        "phases_ms": {key: round(avg(key), 3) for key in
                      ("t_validate_ms", "t_update_ms", "t_merge_ms", "t_sssp_ms", "t_pr_ms", "t_total_ms")},
        "per_batch": {"pr_iterations": avg("pr_iterations"), "pr_affected": avg("pr_affected"),
                      "sssp_invalidated": avg("sssp_invalidated"), "sssp_steps": avg("sssp_steps"),
                      "deleted": avg("deleted"), "inserted": avg("inserted"), "merged": sum(x["merged"] for x in stats)},
        "gteps": round(sum(x["edges_traversed"] for x in stats) / elapsed / 1e9, 3),
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)
    G.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
