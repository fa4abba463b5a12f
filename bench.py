#!/usr/bin/env python3
"""Dynamic-graph update throughput on one MI355X.

Default workload (one step): a batch of updates (default 100,000: half
deletions of existing arcs, half insertions of new uniform arcs, weights
U[1,100]) applied to a directed R-MAT scale-22 graph (4,194,304 vertices,
67,108,864 arcs, a=0.57 b=0.19 c=0.19, weights U[1,100]) that keeps a
shortest-path query from vertex 0 and a PageRank query (damping 0.85, L1
tolerance 1e-9, FP64) current.  Every step gets its own batch (all drawn against
the initial graph); the batches are resident in HBM before the timed region.
value = updates applied per second of wall time over the timed steps.

Also reported: the static-recompute GPU path on the same graph (batch apply
plus SSSP and PageRank from scratch), the roofline of the dominant kernel from
HIP-event launch timing inside this run, and the CPU oracle (edge-list apply +
Dijkstra + FP64 power iteration) timed on the host for one batch.

Other workloads (--workload), each printing one line of the same form:
  grid     4096 x 4096 4-neighbour grid (weights U[1,1000]) with SSSP + PageRank;
  tc       undirected R-MAT scale 20 (16,777,216 edges) with an exact triangle
           count, batches of --pct of |E|;
  batched  4,096 directed R-MAT graphs (scale U{10..14}, 16 arcs per vertex),
           each with its own batch of U[1%,10%] of its arcs, dynamic SSSP from 0
           of every member in one set update (autotuned);
  serve    64 resident R-MAT graphs (scale U{12..20}), open-loop Poisson request
           arrivals; each request is a batch of log-uniform[100, 1e5] updates
           plus one query (SSSP 40 %, PageRank 40 %, triangles 20 %).
One GPU only.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import re
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "dyn SSSP/PR/TC updates/sec + HBM GB/s vs static recompute; serve p50/p99"
CSRC = os.path.join(ROOT, "paper_2507_11094_amd", "csrc")

# HBM bytes per launch read from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per
# dispatch) for the named kernel and workload, divided by what the same counters
# read per byte of a plain 256 MiB device copy (FETCH_SIZE 0.5, WRITE_SIZE 1.0
# counted bytes per byte moved).  Each entry holds the SHA-1 that kernel_sha1()
# gives for the kernel (its definition, the same file's device functions it calls
# and the constants they use) at the time the counters were taken, and the vertex
# order the graph had (single graphs); a changed kernel or another order makes the
# figure stale and it is reported as null.
MEASURED_TRAFFIC: dict = {
    ("k_pr_tiles", "rmat22-dynamic-sssp+pagerank"): {
        "source": "pagerank.hip", "sha1": "0574e0f730155f07581ee12981ec958cc4f34672", "vertex_order": 0,
        "fetch_kib": 585895.5, "write_kib": 33195.3, "fetch_factor": 0.5, "write_factor": 1.0},
    ("k_pr_tiles", "grid4096x4096-dynamic-sssp+pagerank"): {
        "source": "pagerank.hip", "sha1": "0574e0f730155f07581ee12981ec958cc4f34672", "vertex_order": 0,
        "fetch_kib": 396397.8, "write_kib": 131599.9, "fetch_factor": 0.5, "write_factor": 1.0},
    ("k_merge_tiles", "batched4096-rmat10to14-dynamic-sssp"): {
        "source": "graph.hip", "sha1": "42eb1ae1802d55bcf79c17e2dad7845aa22a545e",
        "fetch_kib": 2160799.4, "write_kib": 3510049.5, "fetch_factor": 0.5, "write_factor": 1.0},
    ("k_tc_delta", "rmat20-undirected-dynamic-tc"): {
        "source": "tc.hip", "sha1": "b5076bb4a16ebdc8ac0ef337fe1ae942a48ca96a", "vertex_order": 0,
        "fetch_kib": 408466.4, "write_kib": 768.0, "fetch_factor": 0.5, "write_factor": 1.0},
}

# Serving objective stated up front: 99th percentile latency (submit -> result
# on the host) at the default arrival rate.
SERVE_SLO_P99_MS = 250.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _body(text: str, i: int) -> tuple:
    """(start, end) of the definition whose signature contains offset i: from the
    line before the signature (a template's parameter line) to the closing brace."""
    start = text.rfind("\n", 0, text.rfind("\n", 0, i)) + 1
    j = text.index("{", i)
    depth = 0
    for k in range(j, len(text)):
        depth += {"{": 1, "}": -1}.get(text[k], 0)
        if depth == 0:
            return start, k + 1
    return start, len(text)


def kernel_sha1(fname: str, kernel: str) -> str:
    """SHA-1 of what a kernel's code is made of in its own source file: its
    definition, the definitions of the same file's device functions it calls, and
    the file's constexpr lines whose names either of those use."""
    with open(os.path.join(CSRC, fname)) as f:
        text = f.read()
    i = text.find(f"void {kernel}(")
    if i < 0:
        return ""
    a, b = _body(text, i)
    parts = [text[a:b]]
    helpers = re.finditer(r"__device__[^;{(]*?\b(\w+)\s*\(", text)
    for m in helpers:
        name = m.group(1)
        if name != kernel and re.search(rf"\b{name}\s*[<(]", parts[0]):
            ha, hb = _body(text, m.start(1))
            parts.append(text[ha:hb])
    used = "\n".join(parts)
    for m in re.finditer(r"^\s*constexpr[^=\n]*?\b(\w+)\s*=[^\n]*$", text, re.M):
        if re.search(rf"\b{m.group(1)}\b", used):
            parts.append(m.group(0).strip())
    return hashlib.sha1("\n".join(parts).encode()).hexdigest()


def traffic_for(kernel: str, workload: str, order=None):
    e = MEASURED_TRAFFIC.get((kernel, workload))
    if not e or kernel_sha1(e["source"], kernel) != e["sha1"] or e.get("vertex_order") != order:
        return None
    return round(e["fetch_kib"] * 1024 / e["fetch_factor"] + e["write_kib"] * 1024 / e["write_factor"])


KERNEL_SOURCE = {"pr_pull": ("k_pr_pull", "pagerank.hip"), "pr_tiles": ("k_pr_tiles", "pagerank.hip"),
                 "pr_apply": ("k_pr_apply", "pagerank.hip"),
                 "merge_base": ("k_merge_tiles", "graph.hip"),
                 "sssp_worklist": ("k_wl_cut + pull + k_wl_push", "worklist.hip"),
                 "tc_delta": ("k_tc_delta", "tc.hip")}


_COPY_GBS = None


def copy_peak_gbs() -> float:
    """Device-to-device copy bandwidth measured here (1 GiB, read + write bytes per
    second, best of 10), reported beside the 8 TB/s vendor peak."""
    global _COPY_GBS
    if _COPY_GBS is None:
        import torch

        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        best = float("inf")
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        _COPY_GBS = round(2 * a.numel() / (best * 1e-3) / 1e9, 1)
        del a, b
        torch.cuda.empty_cache()
    return _COPY_GBS


# What the library's edges_traversed tally covers: adjacency entries examined by
# the PageRank pulls (entries x steps), the SSSP frontier steps (every entry of
# every frontier vertex's row, base and diff level, in the cut walk, the pull and
# the push rounds; the work-queue schedule counts arcs examined) and the triangle
# kernel (entries of the shorter row intersected per changed edge).
GTEPS_COUNTS = ("PageRank pull entries x steps + SSSP frontier-row entries (cut, pull, push) + "
                "triangle shorter-row entries")
# GTEPS as a fraction of the HBM roofline: an examined entry moves at least its
# 4-byte column id and one 8-byte gathered value (the PageRank pull's 12 bytes; an
# SSSP relaxation moves more), so 8 TB/s bounds the rate at 8000 / 12 G entries/s.
GTEPS_BYTES_PER_EDGE = 12.0


def gteps_of(stats, elapsed):
    e = sum(x["edges_traversed"] for x in stats)
    return round(e / elapsed / 1e9, 3) if e > 0 else None


def gteps_roofline(gteps):
    if gteps is None:
        return None
    peak = HBM_PEAK_GBS / GTEPS_BYTES_PER_EDGE
    return {"bytes_per_edge": GTEPS_BYTES_PER_EDGE, "peak_gteps": round(peak, 1), "frac": round(gteps / peak, 4)}


def step_spread(ms: list) -> dict:
    """Median, p10 and p90 of the per-step times (library phase timer)."""
    v = np.asarray(ms, dtype=np.float64)
    return {"median_ms": round(float(np.median(v)), 3), "p10_ms": round(float(np.percentile(v, 10)), 3),
            "p90_ms": round(float(np.percentile(v, 90)), 3)}


def roofline_of(prof: dict, workload: str, prefer: str | None = None, order=None) -> dict | None:
    """Roofline of the dominant profiled kernel (largest total time), or `prefer`."""
    if not prof:
        return None
    name = prefer if prefer in prof else max(prof, key=lambda x: prof[x]["ms"])
    p = prof[name]
    launches = max(p["launches"], 1)
    achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] > 0 else 0.0
    kname = KERNEL_SOURCE.get(name, (name, None))[0]
    copy = copy_peak_gbs()
    traffic = traffic_for(kname, workload, order)
    # HBM bytes the counters saw per launch, over the same launch time
    moved = traffic / (1e-3 * p["ms"] / launches) / 1e9 if traffic and p["ms"] > 0 else None
    return {
        "kernel": kname,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "copy_measured": copy,
        "frac_of_copy": round(achieved / copy, 4) if copy else None,
        "traffic": traffic,
        "traffic_GBs": round(moved, 1) if moved else None,
        "traffic_frac": round(moved / HBM_PEAK_GBS, 4) if moved else None,
        "launches": p["launches"],
        "avg_launch_us": round(1e3 * p["ms"] / launches, 2),
        "alg_bytes_per_launch": round(p["bytes"] / launches),
    }


def kernel_table(prof: dict) -> dict:
    return {name: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2),
                   "total_ms": round(v["ms"], 3),
                   "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 and v["bytes"] > 0 else None}
            for name, v in prof.items()}


def line(args, value, unit, ms_per_step, dtype, config, roofline, cpu, higher=True, **extra) -> dict:
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": higher,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    return out


class EdgeIndex:
    """Sorted (u << 32 | v) keys of a directed edge list with the position of each
    key's edge, to look up the weights of arcs a batch deletes."""

    def __init__(self, src, dst, w):
        k = (src.astype(np.int64) << 32) | dst.astype(np.int64)
        self.order = np.argsort(k, kind="stable")
        self.keys = k[self.order]
        self.w = w

    def weights(self, a, b):
        q = (a.astype(np.int64) << 32) | b.astype(np.int64)
        pos = np.searchsorted(self.keys, q)
        assert np.all(self.keys[np.minimum(pos, self.keys.size - 1)] == q), "arc not in the graph"
        return self.w[self.order[pos]]


def inverse(batch, index: EdgeIndex):
    """The batch that undoes `batch` on the directed graph it was drawn against:
    its deleted arcs re-inserted with their weights, its inserted arcs deleted."""
    bs, bd, bw, bo = batch
    dels = bo == 0
    w = np.zeros(bs.size, np.int32)
    w[dels] = index.weights(bs[dels], bd[dels])
    return bs.copy(), bd.copy(), w, dels.astype(np.uint8)


# ----------------------------------------------------------------------------- one graph

# graphs generated once per process (the R-MAT 22 graph serves three batch sizes)
_GRAPHS: dict = {}


def cached_graph(key, make):
    if key not in _GRAPHS:
        _GRAPHS.clear()
        _GRAPHS[key] = make()
    return _GRAPHS[key]


def run_single(args, kind: str) -> dict:
    import torch

    import graphgen
    import paper_2507_11094_amd as dg

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    t = time.perf_counter()
    undirected = kind == "tc"
    if kind == "rmat":
        n, s, d, w = cached_graph(("rmat", args.scale), lambda: graphgen.c2r_graph(args.scale))
        k, wmax = args.batch, 100
        wl = f"rmat{args.scale}-dynamic-sssp+pagerank"
    elif kind == "grid":
        n, s, d, w = cached_graph(("grid", args.side), lambda: graphgen.c2g_graph(args.side))
        k, wmax = args.batch, 1000
        wl = f"grid{args.side}x{args.side}-dynamic-sssp+pagerank"
    else:
        n, s, d = cached_graph(("tc", args.tc_scale), lambda: graphgen.c3_graph(args.tc_scale))[:3]
        w = None
        k, wmax = int(args.pct * s.size), 100
        wl = f"rmat{args.tc_scale}-undirected-dynamic-tc"
    log(f"{wl}: n={n} m={s.size} ready in {time.perf_counter() - t:.1f}s")
    keys = graphgen.edge_keys(s, d, undirected)
    t = time.perf_counter()
    batches = [graphgen.update_batch(n, s, d, k, graphgen.config_seed(1 if kind != "tc" else 2, 100 + i),
                                     wmax=wmax, undirected=undirected, existing=keys) for i in range(W + K)]
    log(f"{W + K} batches of {k} drawn in {time.perf_counter() - t:.1f}s")
    dbatches = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in b) for b in batches]
    torch.cuda.synchronize()
    # --host-batches: the library copies each batch from host memory inside the timed steps
    ubatches = [tuple(np.ascontiguousarray(x) for x in b) for b in batches] if args.host_batches else dbatches

    persistent = max(args.sssp_persistent, 0)
    delta = args.sssp_delta if args.sssp_delta >= 0 else (8000 if kind == "grid" else 0)
    cfg = dg.Config()
    cfg.heavy_degree = args.heavy_degree
    cfg.sssp_persistent = persistent
    cfg.sssp_delta = delta
    cfg.pr_mode = args.pr_mode
    cfg.pr_pull = args.pr_pull
    cfg.pr_tile = args.pr_tile
    cfg.merge_tile = args.merge_tile
    cfg.vertex_order = args.vertex_order
    cfg.pr_extrapolate = 0 if args.pr_plain else 1
    t = time.perf_counter()
    G = dg.Graph(n, s, d, w, undirected=undirected, config=cfg)
    log(f"graph built on device in {time.perf_counter() - t:.2f}s")
    t = time.perf_counter()
    if kind == "tc":
        qt = G.tc_attach()
        tc0 = qt.read()
    else:
        G.sssp_attach(0)
        G.pr_attach(0.85, 1e-9, 1000)
    log(f"queries attached (static solves) in {time.perf_counter() - t:.2f}s")

    for i in range(W):
        G.apply(*ubatches[i])
        log(f"warmup {i + 1}/{W}")
    info_start = G.info()
    dg.dg_profile_enable(True)
    dg.dg_profile_reset()
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        st = G.apply(*ubatches[W + i])
        stats.append(st.as_dict())
        log(f"step {i + 1}/{K}: {st.t_total_ms:.2f} ms (sssp {st.t_sssp_ms:.2f}, pr {st.t_pr_ms:.2f}, "
            f"tc {st.t_tc_ms:.2f}, update {st.t_update_ms + st.t_validate_ms:.2f}, merge {st.t_merge_ms:.2f}, "
            f"pr_iters {st.pr_iterations} ({st.pr_moves} moves), |A| {st.pr_affected})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = dg.dg_profile_read()
    dg.dg_profile_enable(False)
    value = K * k / elapsed
    info_end = G.info()
    # floor under the pull: the same column stream and gathers with nothing else
    floor_us = G.pr_gather_floor(10) if kind != "tc" else None

    def avg(key):
        return float(np.mean([x[key] for x in stats]))

    # The merge (diff level and tombstones back into plain CSR) runs once the two
    # pass 5 % of the live edges, every few dozen batches, so a short timed window
    # may hold none.  Its cost per batch: one forced merge, timed, spread over the
    # batches that fill the threshold at the growth rate of the timed steps.
    merge = None
    growth = ((info_end["diff_entries"] + info_end["tombstones"]) -
              (info_start["diff_entries"] + info_start["tombstones"])) / K
    merged_in_window = sum(x["merged"] for x in stats)
    if merged_in_window == 0 and growth > 0:
        torch.cuda.synchronize()
        t = time.perf_counter()
        G.merge()
        torch.cuda.synchronize()
        merge_s = time.perf_counter() - t
        arcs_fwd = info_end["m"] * (2 if undirected else 1)
        per_merge = 0.05 * arcs_fwd / growth
        amort = merge_s / per_merge
        merge = {"forced_merge_ms": round(1e3 * merge_s, 3), "fwd_growth_per_batch": round(growth, 1),
                 "batches_per_merge": round(per_merge, 1), "amortised_ms_per_batch": round(1e3 * amort, 4),
                 "value_with_amortised_merge": round(K * k / (elapsed + K * amort), 1)}
        log(f"merge: {merge}")

    static = None
    if not args.no_static:
        t_apply = 1e-3 * (avg("t_validate_ms") + avg("t_update_ms") + avg("t_merge_ms"))
        torch.cuda.synchronize()
        if kind == "tc":
            t = time.perf_counter()
            G.tc_static()
            t_s = time.perf_counter() - t
            static = {"tc_ms": round(1e3 * t_s, 3), "apply_ms": round(1e3 * t_apply, 3)}
        else:
            t = time.perf_counter()
            G.sssp_static(0)
            t_ss = time.perf_counter() - t
            t = time.perf_counter()
            _, it_pr = G.pr_static(0.85, 1e-9, 1000)
            t_ps = time.perf_counter() - t
            t_s = t_ss + t_ps
            static = {"sssp_ms": round(1e3 * t_ss, 3), "pr_ms": round(1e3 * t_ps, 3), "pr_iterations": it_pr,
                      "apply_ms": round(1e3 * t_apply, 3)}
        static["updates_per_s"] = round(k / (t_apply + t_s), 1)
        static["dynamic_speedup"] = round((t_apply + t_s) / (elapsed / K), 3)
        log(f"static recompute: {static}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_single(args, kind, n, s, d, w, batches[W], k)

    config = {"workload": wl, "vertices": n, "arcs": int(s.size) * (2 if undirected else 1),
              "batch": k, "insert_fraction": 0.5, "parallelism": "1 gpu",
              "heavy_degree": args.heavy_degree or 512, "sssp_persistent": persistent, "sssp_delta": delta,
              "pr_mode": args.pr_mode, "pr_steps": "plain Jacobi" if args.pr_plain else "extrapolated Jacobi",
              "vertex_order": ["by degree", "as given"][args.vertex_order],
              "batches_in": "host memory (copied inside the timed steps)" if args.host_batches else "HBM",
              "pr_pull": ["merge-path tiles, non-temporal streams", "vertex waves", "merge-path tiles"][args.pr_pull]}
    if kind == "tc":
        config.update({"undirected_edges": int(s.size), "batch_fraction": args.pct, "queries": ["triangles"]})
    else:
        config["queries"] = ["sssp(0)", "pagerank(0.85, l1 1e-9)"]
    extra = {
        "static_recompute": static,
        "phases_ms": {key: round(avg(key), 3) for key in
                      ("t_validate_ms", "t_update_ms", "t_merge_ms", "t_sssp_ms", "t_pr_ms", "t_tc_ms",
                       "t_total_ms")},
        "per_batch": {"pr_iterations": avg("pr_iterations"), "pr_moves": avg("pr_moves"),
                      "pr_affected": avg("pr_affected"),
                      "sssp_invalidated": avg("sssp_invalidated"), "sssp_steps": avg("sssp_steps"),
                      "deleted": avg("deleted"), "inserted": avg("inserted"),
                      "tc_removed": avg("tc_removed"), "tc_added": avg("tc_added"),
                      "merged": sum(x["merged"] for x in stats)},
        "gteps": gteps_of(stats, elapsed),
        "gteps_roofline": gteps_roofline(gteps_of(stats, elapsed)),
        "gteps_counts": GTEPS_COUNTS,
        "step_ms": step_spread([x["t_total_ms"] for x in stats]),
        "kernels": kernel_table(prof),
    }
    if kind == "tc":
        extra["triangles"] = {"initial": int(tc0), "final": int(qt.read())}
    if merge:
        extra["merge"] = merge
    roof = roofline_of(prof, wl, order=args.vertex_order)
    if roof and roof["kernel"] == "k_pr_tiles" and floor_us:
        roof["gather_floor_us"] = round(floor_us, 2)
        roof["frac_of_gather_floor"] = round(floor_us / roof["avg_launch_us"], 4)
    out = line(args, value, "updates/s", 1e3 * elapsed / K, "u64" if kind == "tc" else "i32+f64", config,
               roof, cpu, **extra)
    G.close()
    return out


def host_facts() -> dict:
    """nproc and CPU model of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


# Dijkstra + power iteration time of the last full-graph oracle sample, by graph:
# the R-MAT 22 lines at 10k and 1M updates reuse it (it does not depend on the
# batch size) and time only their own edge-list apply.
_CPU_RECOMPUTE: dict = {}


def cpu_single(args, kind, n, s, d, w, batch, k):
    import oracle

    if kind == "tc":
        # a full recount at scale 20 takes minutes on one core (about 2.6x per
        # scale step), so the sample is the same recipe at scale <= 17
        import graphgen

        sc = min(args.tc_scale, 17)
        if sc != args.tc_scale:
            n, s, d = graphgen.c3_graph(sc)
            k = int(args.pct * s.size)
            batch = graphgen.update_batch(n, s, d, k, graphgen.config_seed(2, 100), undirected=True)
        t = time.perf_counter()
        s2, d2, _, _ = oracle.apply(n, s, d, None, *batch, undirected=True)
        oracle.triangles(n, s2, d2)
        t_cpu = time.perf_counter() - t
        sample = (f"one {k}-update batch ({args.pct:g} of |E|) on the undirected R-MAT recipe at scale {sc}: "
                  f"edge-list apply and a full triangle recount (single thread)")
    elif kind == "grid":
        # a bounded sample: the same recipe on a quarter-size grid with a quarter of
        # the batch (the full grid's power iteration alone takes about half a minute)
        import graphgen

        side = min(args.side, 2048)
        kk = max(2, k * side * side // (args.side * args.side))
        if side != args.side:
            n, s, d, w = graphgen.c2g_graph(side)
            batch = graphgen.update_batch(n, s, d, kk, graphgen.config_seed(1, 100), wmax=1000)
        t = time.perf_counter()
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *batch)
        oracle.sssp(n, s2, d2, w2, 0)
        oracle.pagerank(n, s2, d2, 0.85, 1e-9, 1000)
        t_cpu = time.perf_counter() - t
        k = kk
        sample = (f"one {kk}-update batch on the {side}x{side} grid recipe: edge-list apply, Dijkstra from 0, "
                  f"FP64 power iteration to L1 1e-9 (single thread)")
    else:
        key = (kind, args.scale)
        t = time.perf_counter()
        s2, d2, w2, _ = oracle.apply(n, s, d, w, *batch)
        t_apply = time.perf_counter() - t
        if key in _CPU_RECOMPUTE:
            t_cpu = t_apply + _CPU_RECOMPUTE[key]
            sample = (f"one {k}-update batch on the full graph: edge-list apply timed "
                      f"({t_apply:.2f} s), plus the Dijkstra from 0 and FP64 power iteration time of the "
                      f"100k-update sample on the same graph (single thread)")
        else:
            t = time.perf_counter()
            oracle.sssp(n, s2, d2, w2, 0)
            oracle.pagerank(n, s2, d2, 0.85, 1e-9, 1000)
            t_re = time.perf_counter() - t
            _CPU_RECOMPUTE[key] = t_re
            t_cpu = t_apply + t_re
            sample = (f"one {k}-update batch on the full graph: edge-list apply, Dijkstra from 0, FP64 power "
                      f"iteration to L1 1e-9 (single thread)")
    log(f"cpu oracle: {t_cpu:.1f}s")
    return {"value": round(k / t_cpu, 1), "unit": "updates/s", "cores": 1, "kind": "oracle",
            "seconds": round(t_cpu, 2), "sample": sample, **host_facts()}


# ----------------------------------------------------------------------------- batched set

def set_members(count: int, seed: int):
    """Member graphs of the batched workload: scale U{10..14}, 16 arcs per vertex,
    batch sizes U[1 %, 10 %] of each member's arcs."""
    import graphgen

    scales = graphgen.uniform_int(graphgen.stream_seed(seed, "scale"), 0, count, 10, 14)
    frac = 0.01 + 0.09 * graphgen.uniform01(graphgen.stream_seed(seed, "frac"), 0, count)
    members, ks = [], []
    for i in range(count):
        sc = int(scales[i])
        members.append(graphgen.rmat_directed(sc, 16 << sc, graphgen.config_seed(3, i)))
        ks.append(int(frac[i] * (16 << sc)))
        if (i + 1) % 1024 == 0:
            log(f"  {i + 1}/{count} members")
    return members, ks


def run_batched(args) -> dict:
    import torch

    import graphgen
    import paper_2507_11094_amd as dg

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    count = args.graphs or 4096
    t = time.perf_counter()
    members, ks = set_members(count, graphgen.config_seed(3, 0))
    log(f"{count} members generated in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    fwd, bwd = [], []
    for i, ((n, s, d, w), k) in enumerate(zip(members, ks)):
        idx = EdgeIndex(s, d, w)
        fwd.append(graphgen.update_batch(n, s, d, k, graphgen.config_seed(3, 100000 + i), existing=idx.keys))
        bwd.append(inverse(fwd[-1], idx))
    log(f"batches drawn in {time.perf_counter() - t:.1f}s (forward + inverse)")
    total_k = int(sum(ks))

    def concat(bs):
        kk = np.array([b[0].size for b in bs], np.int64)
        cols = [torch.from_numpy(np.ascontiguousarray(np.concatenate([b[j] for b in bs]))).to(dev)
                for j in range(4)]
        return kk, cols

    dfwd, dbwd = concat(fwd), concat(bwd)
    torch.cuda.synchronize()
    cfg = dg.Config()
    cfg.heavy_degree = args.heavy_degree
    cfg.merge_tile = args.merge_tile
    t = time.perf_counter()
    S = dg.GraphSet(members, config=cfg)
    info = S.info()
    log(f"set built: {info} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    S.sssp_attach(np.zeros(count, np.int32))
    log(f"sssp attached (static multi-source solve) in {time.perf_counter() - t:.2f}s")
    tune = None
    if not args.no_autotune:
        t = time.perf_counter()
        best, best_ms = S.autotune(fwd)
        tune = {"heavy_degree": best.heavy_degree, "persistent_groups": best.persistent_groups,
                "best_ms": round(best_ms, 3), "seconds": round(time.perf_counter() - t, 1)}
        log(f"autotune: {tune}")
    # steps alternate the forward batches and their inverses: every step is a
    # genuine 50/50 batch against the graph it meets
    for i in range(W):
        kk, cols = dfwd if i % 2 == 0 else dbwd
        S.apply_device(kk, *cols)
    dg.dg_profile_enable(True)
    dg.dg_profile_reset()
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        kk, cols = dfwd if (W + i) % 2 == 0 else dbwd
        st = S.apply_device(kk, *cols)
        stats.append(st.as_dict())
        log(f"step {i + 1}/{K}: {st.t_total_ms:.2f} ms (sssp {st.t_sssp_ms:.2f}, update "
            f"{st.t_update_ms + st.t_validate_ms:.2f}, merge {st.t_merge_ms:.2f}, cut {st.sssp_invalidated})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = dg.dg_profile_read()
    dg.dg_profile_enable(False)
    gstats = S.graph_stats()

    static = None
    if not args.no_static:
        # static comparator: a fresh set (the initial graphs), the forward batches
        # applied, then every member's SSSP from scratch
        kk, cols = dfwd
        cfg2 = dg.Config()
        cfg2.merge_tile = args.merge_tile
        S2 = dg.GraphSet(members, config=cfg2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = S2.apply_device(kk, *cols)
        torch.cuda.synchronize()
        t_a = time.perf_counter() - t
        S2.sssp_attach(np.zeros(count, np.int32))
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t
        static = {"ms": round(1e3 * t_s, 3), "apply_ms": round(1e3 * t_a, 3),
                  "sssp_ms": round(1e3 * (t_s - t_a), 3), "updates_per_s": round(total_k / t_s, 1),
                  "dynamic_speedup": round(t_s / (elapsed / K), 3)}
        S2.close()
        log(f"static recompute: {static}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        sample = min(count, args.cpu_members)
        t = time.perf_counter()
        upd = 0
        for i in range(sample):
            n, s, d, w = members[i]
            s2, d2, w2, _ = oracle.apply(n, s, d, w, *fwd[i])
            oracle.sssp(n, s2, d2, w2, 0)
            upd += ks[i]
        t_cpu = time.perf_counter() - t
        cpu = {"value": round(upd / t_cpu, 1), "unit": "updates/s", "cores": 1, "kind": "oracle",
               "seconds": round(t_cpu, 2),
               "sample": f"the first {sample} members of the set: edge-list apply of each member's batch and "
                         f"Dijkstra from 0 (single thread)", **host_facts()}
        log(f"cpu oracle: {cpu}")

    def avg(key):
        return float(np.mean([x[key] for x in stats]))

    config = {"workload": f"batched{count}-rmat10to14-dynamic-sssp", "graphs": count,
              "vertices": info["vertices"], "arcs": info["arcs"], "updates_per_step": total_k,
              "batch_fraction": "U[0.01,0.10] per member", "insert_fraction": 0.5, "queries": ["sssp(0) per member"],
              "parallelism": "1 gpu", "autotune": tune}
    out = line(args, K * total_k / elapsed, "updates/s", 1e3 * elapsed / K, "i32", config,
               roofline_of(prof, config["workload"], "sssp_worklist"), cpu,
               static_recompute=static,
               phases_ms={key: round(avg(key), 3) for key in
                          ("t_validate_ms", "t_update_ms", "t_merge_ms", "t_sssp_ms", "t_total_ms")},
               per_step={"sssp_invalidated": avg("sssp_invalidated"), "deleted": avg("deleted"),
                         "inserted": avg("inserted"), "merged": sum(x["merged"] for x in stats)},
               gteps=gteps_of(stats, elapsed), gteps_roofline=gteps_roofline(gteps_of(stats, elapsed)),
               gteps_counts=GTEPS_COUNTS,
               step_ms=step_spread([x["t_total_ms"] for x in stats]),
               graph_launches=gstats, kernels=kernel_table(prof))
    S.close()
    return out


# ----------------------------------------------------------------------------- serving

def serve_graphs(count: int, seed: int):
    import graphgen

    scales = graphgen.uniform_int(graphgen.stream_seed(seed, "scale"), 0, count, 12, 20)
    out = []
    for i, sc in enumerate(scales):
        out.append(graphgen.rmat_directed(int(sc), 16 << int(sc), graphgen.config_seed(4, i)))
        if (i + 1) % 16 == 0:
            log(f"  {i + 1}/{count} graphs")
    return out


def serve_requests(graphs, seed: int, rate: float, duration: float):
    """Open-loop request stream: Poisson arrivals, graph uniform, batch size
    log-uniform in [100, 1e5], query kinds 40/40/20, source uniform.  For each
    graph its requests alternate a fresh batch and that batch's inverse, so every
    batch is drawn against the graph it will meet."""
    import graphgen

    count = int(rate * duration * 1.5) + 16
    gaps = -np.log(1.0 - graphgen.uniform01(graphgen.stream_seed(seed, "gap"), 0, count)) / rate
    at = np.cumsum(gaps)
    count = int(np.searchsorted(at, duration))
    gi = graphgen.uniform_int(graphgen.stream_seed(seed, "graph"), 0, count, 0, len(graphs) - 1)
    ku = graphgen.uniform01(graphgen.stream_seed(seed, "k"), 0, count)
    qu = graphgen.uniform01(graphgen.stream_seed(seed, "kind"), 0, count)
    su = graphgen.uniform01(graphgen.stream_seed(seed, "source"), 0, count)
    index = {}
    pending_inverse = {}
    reqs = []
    for i in range(count):
        g = int(gi[i])
        n, s, d, w = graphs[g]
        if g in pending_inverse:
            b = pending_inverse.pop(g)
        else:
            k = int(round(np.exp(np.log(100) + ku[i] * (np.log(1e5) - np.log(100)))))
            k = min(k, s.size)  # never more deletions than half the graph's arcs
            if g not in index:
                index[g] = EdgeIndex(s, d, w)
            b = graphgen.update_batch(n, s, d, k, graphgen.config_seed(4, 10000 + i), existing=index[g].keys)
            pending_inverse[g] = inverse(b, index[g])
        kind = 0 if qu[i] < 0.4 else (1 if qu[i] < 0.8 else 2)
        if (i + 1) % 100 == 0:
            log(f"  {i + 1}/{count} requests drawn")
        reqs.append((float(at[i]), g, kind, int(su[i] * n), b))
    return reqs


def run_serve(args) -> dict:
    import torch

    import graphgen
    import paper_2507_11094_amd as dg

    count = args.graphs or 64
    seed = graphgen.config_seed(4, 0)
    t = time.perf_counter()
    graphs = serve_graphs(count, seed)
    log(f"{count} graphs generated in {time.perf_counter() - t:.1f}s "
        f"({sum(g[0] for g in graphs)} vertices, {sum(g[1].size for g in graphs)} arcs)")
    t = time.perf_counter()
    reqs = serve_requests(graphs, seed, args.rate, args.duration)
    log(f"{len(reqs)} requests drawn in {time.perf_counter() - t:.1f}s")
    S = dg.Server(workers=args.workers, budget_bytes=args.budget_gib << 30)
    t = time.perf_counter()
    gcfg = None
    if args.diff_only:
        gcfg = dg.Config()
        gcfg.diff_only = 1
    for n, s, d, w in graphs:
        S.add_graph(n, s, d, w, config=gcfg)
    torch.cuda.synchronize()
    log(f"graphs resident in {time.perf_counter() - t:.1f}s")
    S.start()
    # warmup: one request per kind on graph 0 (and its inverse), untimed
    n0, s0, d0, w0 = graphs[0]
    idx0 = EdgeIndex(s0, d0, w0)
    wb = graphgen.update_batch(n0, s0, d0, 1000, graphgen.config_seed(4, 999), existing=idx0.keys)
    wi = inverse(wb, idx0)
    for kind, b in ((0, wb), (1, wi), (2, wb), (1, wi)):
        S.wait(S.submit(0, kind, *b, source=0))

    tickets = []
    lock = threading.Lock()
    results = []
    done = threading.Event()

    def collector():
        i = 0
        while True:
            with lock:
                if i >= len(tickets):
                    if done.is_set():
                        return
                    tk = None
                else:
                    tk = tickets[i]
            if tk is None:
                time.sleep(0.0005)
                continue
            res, _ = S.wait(tk[0])
            results.append((tk[1], res.status, res.t_submit, res.t_start, res.t_end, tk[2]))
            if res.status != 0:
                log(f"request {i} (kind {tk[1]}, {tk[2]} updates) failed: [{res.status}] "
                    f"{res.error.decode(errors='replace')}")
            i += 1

    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    for at, g, kind, source, b in reqs:
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        tk = S.submit(g, kind, *b, source=source)
        with lock:
            tickets.append((tk, kind, b[0].size))
    done.set()
    th.join()
    elapsed = time.perf_counter() - t0
    S.close()
    bad = [r for r in results if r[1] != 0]
    lat = np.array([1e3 * (r[4] - r[2]) for r in results])
    qwait = np.array([1e3 * (r[3] - r[2]) for r in results])
    upd = int(sum(r[5] for r in results))
    by_kind = {}
    for kname, kv in (("sssp", 0), ("pagerank", 1), ("triangles", 2)):
        l = np.array([1e3 * (r[4] - r[2]) for r in results if r[0] == kv])
        if l.size:
            by_kind[kname] = {"count": int(l.size), "p50_ms": round(float(np.percentile(l, 50)), 3),
                              "p99_ms": round(float(np.percentile(l, 99)), 3)}
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    log(f"served {len(results)} requests in {elapsed:.1f}s: p50 {p50:.1f} ms p99 {p99:.1f} ms, errors {len(bad)}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        t = time.perf_counter()
        upd_c, done_c = 0, 0
        for at, g, kind, source, b in reqs:
            n, s, d, w = graphs[g]
            s2, d2, w2, _ = oracle.apply(n, s, d, w, *b)
            if kind == 0:
                oracle.sssp(n, s2, d2, w2, source)
            elif kind == 1:
                oracle.pagerank(n, s2, d2, 0.85, 1e-9, 1000)
            else:
                u, v = oracle.symmetrise(s2, d2)
                oracle.triangles(n, u, v)
            upd_c += b[0].size
            done_c += 1
            if time.perf_counter() - t > args.cpu_seconds:
                break
        t_cpu = time.perf_counter() - t
        cpu = {"value": round(upd_c / t_cpu, 1), "unit": "updates/s", "cores": 1, "kind": "oracle",
               "seconds": round(t_cpu, 2),
               "sample": f"the first {done_c} requests of the stream, each: edge-list apply against the "
                         f"graph's initial state and a full recompute of its query (single thread)", **host_facts()}
        log(f"cpu oracle: {cpu}")

    config = {"workload": f"serve{count}-rmat12to20-poisson", "graphs": count,
              "vertices": int(sum(g[0] for g in graphs)), "arcs": int(sum(g[1].size for g in graphs)),
              "rate_per_s": args.rate, "duration_s": args.duration, "requests": len(results),
              "batch": "log-uniform[100, 1e5]", "insert_fraction": 0.5,
              "query_mix": {"sssp": 0.4, "pagerank": 0.4, "triangles": 0.2}, "workers": args.workers,
              "budget_gib": args.budget_gib, "parallelism": "1 gpu"}
    out = line(args, upd / elapsed, "updates/s", 1e3 * elapsed / max(len(results), 1), "i32+f64+u64", config,
               None, cpu, serve={"p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
                                 "p99_queue_ms": round(float(np.percentile(qwait, 99)), 3),
                                 "slo_p99_ms": SERVE_SLO_P99_MS, "slo_met": bool(p99 <= SERVE_SLO_P99_MS),
                                 "errors": len(bad), "by_kind": by_kind})
    out["steps"] = len(results)
    out["warmup"] = 4
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat", choices=["rmat", "grid", "tc", "batched", "serve"])
    ap.add_argument("--scale", type=int, default=22, help="rmat: R-MAT scale")
    ap.add_argument("--side", type=int, default=4096, help="grid: side length")
    ap.add_argument("--tc-scale", type=int, default=20, help="tc: R-MAT scale")
    ap.add_argument("--batch", type=int, default=100_000, help="rmat/grid: updates per batch")
    ap.add_argument("--pct", type=float, default=0.01, help="tc: batch size as a fraction of |E|")
    ap.add_argument("--graphs", type=int, default=0, help="batched/serve: member graphs (0: 4096 / 64)")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--duration", type=float, default=15.0, help="serve: seconds of arrivals")
    ap.add_argument("--workers", type=int, default=4, help="serve: worker streams")
    ap.add_argument("--budget-gib", type=int, default=64, help="serve: device-memory admission budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="rmat: skip the other configurations (reported under \"workloads\" by default)")
    ap.add_argument("--cpu-members", type=int, default=256, help="batched: members in the oracle sample")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="serve: seconds of oracle sample")
    ap.add_argument("--no-static", action="store_true")
    ap.add_argument("--host-batches", action="store_true",
                    help="hand the library host arrays (copied over PCIe inside the timed steps) instead of "
                         "batches already in HBM")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--heavy-degree", type=int, default=0, help="rows longer than this are split (0: library default)")
    ap.add_argument("--sssp-persistent", type=int, default=0,
                    help="1: SSSP on the single-launch work queue, 0: frontier steps")
    ap.add_argument("--sssp-delta", type=int, default=-1,
                    help="near-far bucket width of the frontier SSSP (0: plain rounds; -1: grid 8000, else 0)")
    ap.add_argument("--pr-mode", type=int, default=0, help="PageRank form after a batch: 0 auto, 1 local, 2 global")
    ap.add_argument("--pr-pull", type=int, default=0,
                    help="whole-graph PageRank pull: 0 merge-path tiles with non-temporal streams, 1 per-vertex "
                         "waves, 2 merge-path tiles without the hints")
    ap.add_argument("--pr-tile", type=int, default=0, help="rows + entries per pull tile: 1024, 2048 (0) or 4096")
    ap.add_argument("--merge-tile", type=int, default=0,
                    help="rows + entries per merge-path tile of the CSR merge: 512, 1024 or 2048 (0)")
    ap.add_argument("--diff-only", action="store_true",
                    help="serve: new edges always go to the diff level (no reuse of tombstoned slots)")
    ap.add_argument("--pr-plain", action="store_true",
                    help="plain Jacobi PageRank steps (default: extrapolated steps, same stopping rule)")
    ap.add_argument("--vertex-order", type=int, default=0,
                    help="vertex order inside the library: 0 by degree (default), 1 as given")
    ap.add_argument("--gather-ladder", action="store_true",
                    help="only time scattered 8-byte gathers over working sets from 64 KiB to 1 GiB "
                         "(dg_calibrate kind 3) and print the rates")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run five plain 256 MiB device-to-device copies (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale) and exit")
    args = ap.parse_args()
    if args.gather_ladder:
        # Rate of scattered 8-byte gathers against the size of the set they hit: the
        # library's calibration kind 3 (2^26 reads at hashed positions) over working
        # sets from 64 KiB (cache-resident) to 1 GiB (HBM), HIP events on the stream.
        import torch

        import paper_2507_11094_amd as dg

        lib = dg.load_library()
        big = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda:0")
        st = torch.cuda.current_stream()
        rows = []
        for ws_bytes in (64 << 10, 512 << 10, 4 << 20, 32 << 20, 256 << 20, 1 << 30):
            dg._check(lib.dg_calibrate(3, ctypes.c_void_p(big.data_ptr()), ws_bytes, ctypes.c_void_p(st.cuda_stream)))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record(st)
            for _ in range(reps):
                dg._check(lib.dg_calibrate(3, ctypes.c_void_p(big.data_ptr()), ws_bytes,
                                           ctypes.c_void_p(st.cuda_stream)))
            e1.record(st)
            e1.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / reps
            rows.append({"working_set_bytes": ws_bytes, "us_per_launch": round(us, 2),
                         "G_gathers_per_s": round((1 << 26) / us * 1e-3, 1)})
            log(f"gather ladder: {rows[-1]}")
        print(json.dumps({"gather_ladder": rows, "gathers_per_launch": 1 << 26, "bytes_per_gather": 8}), flush=True)
        return 0
    if args.calibrate_copy:
        # Known-traffic launches for scaling the FETCH_SIZE / WRITE_SIZE counters:
        # five plain 256 MiB device copies (torch), then the library's calibration
        # kernels on a 1 GiB buffer: a stream read, a stream write and a gather of
        # one word per 128-byte line (8 Mi lines).
        import torch

        import paper_2507_11094_amd as dg

        a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        big = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        lib = dg.load_library()
        for kind in (0, 1, 2):
            for _ in range(3):
                dg._check(lib.dg_calibrate(kind, ctypes.c_void_p(big.data_ptr()), big.numel(), None))
        print(json.dumps({"calibrate_copy_bytes": 256 << 20, "copies": 5, "calibrate_kernel_bytes": 1 << 30,
                          "kernels": {"k_cal_read": "reads 1 GiB", "k_cal_write": "writes 1 GiB",
                                      "k_cal_gather": "reads one word of each of 8 Mi 128-byte lines"}}),
              flush=True)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the dynamic-graph hot path on one MI355X, so --gpus must be 1; "
              "sharding over several GPUs is designed (vertex partition, RCCL exchanges) but not built.",
              file=sys.stderr)
        return 2
    if args.workload in ("rmat", "grid", "tc"):
        out = run_single(args, args.workload)
    elif args.workload == "batched":
        out = run_batched(args)
    else:
        out = run_serve(args)
    if args.workload == "rmat" and not args.no_workloads:
        out["workloads"] = run_workloads(args)
    print(json.dumps(out), flush=True)
    return 0


# The other configurations, each measured in the same run with fewer steps and a
# bounded oracle sample, reported under "workloads" of the R-MAT 22 line.
WORKLOADS = [
    ("rmat22-10k", "rmat", {"batch": 10_000, "steps": 10, "warmup": 3}),
    ("rmat22-1M", "rmat", {"batch": 1_000_000, "steps": 5, "warmup": 2}),
    ("grid4096-100k", "grid", {"batch": 100_000, "steps": 5, "warmup": 2}),
    ("tc-rmat20-1pct", "tc", {"pct": 0.01, "steps": 10, "warmup": 3}),
    ("batched4096", "batched", {"steps": 4, "warmup": 2, "cpu_members": 64}),
    ("serve64", "serve", {"duration": 10.0, "rate": 20.0, "cpu_seconds": 8.0}),
]
# keys of a workload line that repeat the R-MAT 22 line's
_SHARED = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")


def run_workloads(args) -> dict:
    import copy

    out = {}
    for name, kind, over in WORKLOADS:
        a = copy.copy(args)
        for key, v in over.items():
            setattr(a, key, v)
        if kind in ("rmat", "grid"):
            a.sssp_delta = -1  # the grid's near-far default
        log(f"---- workload {name}")
        t = time.perf_counter()
        if kind in ("rmat", "grid", "tc"):
            res = run_single(a, kind)
        elif kind == "batched":
            res = run_batched(a)
        else:
            res = run_serve(a)
        res = {key: v for key, v in res.items() if key not in _SHARED}
        res["wall_s"] = round(time.perf_counter() - t, 1)
        out[name] = res
    return out


if __name__ == "__main__":
    sys.exit(main())
