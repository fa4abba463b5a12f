// Single-source shortest paths: static solve and the dynamic update.
//
// State per query: key[v] = (dist << 32) | parent as one 64-bit word, so the
// Min construct of the Dynamic SSSP listing of Appendix A (distance, modified
// flag and parent updated together) is a single atomicMin; ties in distance
// resolve to the smaller parent id, and any tie is a valid tree.  Distances
// saturate at INF: a vertex whose shortest distance is INF or more reads as
// unreachable (INF, parent -1) and is never expanded, which leaves every other
// distance exact because weights are positive.
//
// Dynamic update for one batch (Appendix A, DynSSSP: OnDelete, updateCSRDel,
// Decremental, OnAdd, updateCSRAdd, Incremental), scheduled for a GPU:
//   pre-hook  (old graph)  OnDelete: a deleted arc (u, v) with parent[v] == u cuts
//                          v from the tree: v := (INF, -1).
//   post-hook (new graph)  1. Decremental, phase 1: every vertex whose parent was
//                             cut is cut too -- a frontier walk down the tree edges
//                             instead of the listing's repeated full sweeps.
//                          2. Decremental, phase 2: each cut vertex pulls
//                             min(dist[u] + w) over its live in-edges once.
//                          3. OnAdd: each inserted arc (u, v, w) relaxes v.
//                          4. Incremental: push relaxation to a fixed point from
//                             every vertex whose distance dropped in 2-3.
// Why this reaches the static result: after step 1 every value is the length of a
// path that still exists (uncut vertices keep their old tree path, and deletions
// only lengthen paths), so all values are upper bounds; steps 2-4 then run
// Bellman-Ford from every vertex that could violate d[v] <= d[u] + w, and the fixed
// point of a Bellman-Ford started from achievable upper bounds and all possibly
// violated edges is the exact distance (Section 3.1: only the affected part moves).
#include <algorithm>
#include <cstring>
#include <functional>
#include <vector>

#include "traverse.h"

namespace dg {

// ---- ops for the expansion kernel ---------------------------------------------

// Push relaxation: payload = dist of the frontier vertex.
struct RelaxOp {
    uint64_t *key;
    int32_t *stamp;
    int32_t st;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t v, int32_t &pay) const {
        int32_t d = sssp_dist(__atomic_load_n(&key[v], __ATOMIC_RELAXED));
        pay = d;
        return d < INF;
    }
    __device__ bool edge(bool valid, int32_t v, int32_t d, int32_t x, int32_t w) const {
        bool push = false;
        if (valid) {
            uint64_t cand = sssp_pack(d + w, v);
            // keys only decrease, so a stale plain load can only make us skip a
            // candidate that would not have won the atomicMin either
            if (cand < __atomic_load_n(&key[x], __ATOMIC_RELAXED)) {
                uint64_t old = atomicMin((unsigned long long *)&key[x], (unsigned long long)cand);
                if (cand < old && sssp_dist(cand) < sssp_dist(old))
                    push = atomicExch(&stamp[x], st) != st;
            }
        }
        return push;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

// Decremental phase 1: cut children whose tree parent is the frontier vertex.
struct CutOp {
    uint64_t *key;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t, int32_t &pay) const { pay = 0; return true; }
    __device__ bool edge(bool valid, int32_t v, int32_t, int32_t x, int32_t) const {
        bool cut = false;
        if (valid) {
            uint64_t k = key[x];
            if (sssp_parent(k) == v) {
                key[x] = sssp_pack(INF, -1);
                cut = true;
            }
        }
        return cut;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

// Decremental phase 2: pull over in-edges (reverse store); the frontier holds the
// cut vertices, an edge (v <- x) offers dist[x] + w to v.
struct PullOp {
    uint64_t *key;
    __device__ bool vtx(int32_t, int32_t &pay) const { pay = 0; return true; }
    __device__ bool edge(bool valid, int32_t v, int32_t, int32_t x, int32_t w) const {
        if (!valid) return false;
        int32_t dx = sssp_dist(__atomic_load_n(&key[x], __ATOMIC_RELAXED));
        if (dx >= INF) return false;
        atomicMin((unsigned long long *)&key[v], (unsigned long long)sssp_pack(dx + w, x));
        return false;
    }
    __device__ SinkTarget sink() const { return SinkTarget{}; }
};

// ---- plain kernels ---------------------------------------------------------------

__global__ void k_sssp_init(int32_t n, uint64_t *key, int32_t source) {
    for (int64_t v = gtid(); v < n; v += gstride()) key[v] = sssp_pack(v == source ? 0 : INF, -1);
}

// OnDelete: (u, v) deleted and parent[v] == u  ->  v := (INF, -1), v is a seed.
__global__ void k_sssp_on_delete(int64_t na, const int32_t *adu, const int32_t *adv, uint64_t *key,
                                 int32_t *seeds, int64_t *count) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool cut = false;
        int32_t v = 0;
        if (i < na) {
            v = adv[i];
            if (sssp_parent(key[v]) == adu[i]) {
                key[v] = sssp_pack(INF, -1);
                cut = true;
            }
        }
        int64_t slot = block_append(count, cut, sc);
        if (cut) seeds[slot] = v;
    }
}

// After the pull: cut vertices that now have a finite distance start the push.
__global__ void k_sssp_pulled(int64_t nc, const int32_t *cut, const uint64_t *key, int32_t *stamp,
                              int32_t st, int32_t *front, int64_t *count) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < nc) {
            v = cut[i];
            p = sssp_dist(key[v]) < INF && atomicExch(&stamp[v], st) != st;
        }
        int64_t slot = block_append(count, p, sc);
        if (p) front[slot] = v;
    }
}

// OnAdd: each inserted arc relaxes its head once; improved heads join the push.
__global__ void k_sssp_on_add(int64_t na, const int32_t *aiu, const int32_t *aiv, const int32_t *aiw,
                              uint64_t *key, int32_t *stamp, int32_t st, int32_t *front,
                              int64_t *count) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < na) {
            int32_t u = aiu[i];
            v = aiv[i];
            int32_t du = sssp_dist(key[u]);
            if (du < INF) {
                uint64_t cand = sssp_pack(du + aiw[i], u);
                uint64_t old = atomicMin((unsigned long long *)&key[v], (unsigned long long)cand);
                if (cand < old && sssp_dist(cand) < sssp_dist(old)) p = atomicExch(&stamp[v], st) != st;
            }
        }
        int64_t slot = block_append(count, p, sc);
        if (p) front[slot] = v;
    }
}

// Distances and parents in the caller's ids: vertex v reads internal slot perm[v]
// and a parent id p comes back as iperm[p] (both null when the ids are kept).
__global__ void k_sssp_unpack(int32_t n, const uint64_t *key, const int32_t *perm, const int32_t *iperm,
                              int32_t *dist, int32_t *parent) {
    for (int64_t v = gtid(); v < n; v += gstride()) {
        uint64_t k = key[perm ? perm[v] : v];
        int32_t d = sssp_dist(k);
        if (dist) dist[v] = d >= INF ? INF : d;
        if (parent) {
            const int32_t p = sssp_parent(k);
            parent[v] = d >= INF ? -1 : (iperm && p >= 0 ? iperm[p] : p);
        }
    }
}

// ---- host drivers -------------------------------------------------------------------

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

static int heavy_deg(dg_graph *g) { return g->cfg.heavy_degree > 0 ? g->cfg.heavy_degree : 512; }

// Frontier buffers sized for the graph (n vertices; heavy queue for m / chunk).
static int ensure_frontiers(dg_graph *g) {
    Work &ws = g->ws;
    DG_TRY(ws.f0.ensure((size_t)g->n + 1));
    DG_TRY(ws.f1.ensure((size_t)g->n + 1));
    int64_t edges = g->fwd.m + g->fwd.dm;
    if (g->rev != &g->fwd) edges = std::max(edges, g->rev->m + g->rev->dm);
    DG_TRY(ws.heavy.ensure((size_t)(2 * (edges / heavy_deg(g) + 2) + g->n / 8 + 64) * 2));
    return DG_OK;
}

static ExpandArgs make_args(dg_graph *g, const Dir &d, const int32_t *F, int64_t nf) {
    ExpandArgs a;
    a.F = F;
    a.nf = nf;
    a.g = view(d);
    a.hq = reinterpret_cast<int64_t *>(g->ws.heavy.p);
    a.hcount = g->ws.dcnt + C_HEAVY;
    a.heavy_deg = heavy_deg(g);
    a.chunk = a.heavy_deg;
    // No row longer than the heavy degree (the host copy of the bound, at most one
    // update old): every row is walked in place and the chunk kernel is skipped.  A
    // stale bound only costs time -- a row that grew past it is walked by one wave.
    if (g->ws.hcnt[C_MAXROW] <= (int64_t)a.heavy_deg) a.heavy_deg = NO_HEAVY;
    return a;
}

// The traversal tally (GTEPS) counts the adjacency entries (base + diff,
// tombstones included) of the rows each frontier step walks: the expansion adds
// them up itself when its `tally` argument is set (with_tally).
static ExpandArgs with_tally(ExpandArgs a, int64_t *tally) {
    a.tally = tally;
    return a;
}

// ---- near-far schedule --------------------------------------------------------------
// The push relaxes in Bellman-Ford rounds; on high-diameter graphs with spread
// weights (road networks) a vertex is improved many times before its distance
// settles.  The near-far schedule (Davidson, Baxter, Garland and Owens, IPDPS
// 2014; a two-bucket form of Meyer and Sanders' delta-stepping) relaxes only the
// improved vertices below a threshold T; the others wait in a far pile (each
// vertex at most once, marked by a per-call stamp).  When the near side is empty,
// T moves to (smallest live far distance) + delta and the far pile is split again.
// Far entries below the previous T were relaxed when they dropped below it, so
// they are stale and leave the pile.  Only the order of relaxations changes; the
// fixed point is the same.

// Improved vertices (count on the device) -> near (dist < T) or the far pile.
__global__ void k_nf_split(const int64_t *nn_p, const int32_t *N, const uint64_t *key, int32_t T, int32_t *near,
                           int64_t *nnear, int32_t *far, int64_t *nfar, int32_t *farflag, int32_t fst) {
    __shared__ BlockScratch sc;
    const int64_t nn = *nn_p;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nn; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        bool pn = false, pf = false;
        int32_t v = 0;
        if (i < nn) {
            v = N[i];
            pn = sssp_dist(key[v]) < T;
            pf = !pn && atomicExch(&farflag[v], fst) != fst;
        }
        const int64_t sn = block_append(nnear, pn, sc);
        if (pn) near[sn] = v;
        const int64_t sf = block_append(nfar, pf, sc);
        if (pf) far[sf] = v;
    }
}

// Smallest distance >= T in the far pile, as INF - d through a max (0: none).
__global__ void k_nf_min(int64_t nf, const int32_t *far, const uint64_t *key, int32_t T, int64_t *out) {
    int64_t best = 0;
    for (int64_t i = gtid(); i < nf; i += gstride()) {
        const int32_t d = sssp_dist(key[far[i]]);
        if (d >= T && d < INF) best = max(best, (int64_t)(INF - d));
    }
    best = wave_max_i32((int32_t)best);
    if (lane_id() == 0 && best > 0) atomicMax((unsigned long long *)out, (unsigned long long)best);
}

// Next bucket: entries in [T0, T1) go near, entries >= T1 stay, the rest are stale.
__global__ void k_nf_refill(int64_t nf, const int32_t *far, const uint64_t *key, int32_t T0, int32_t T1,
                            int32_t *near, int64_t *nnear, int32_t *far2, int64_t *nfar2, int32_t *farflag) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        bool pn = false, pk = false;
        int32_t v = 0;
        if (i < nf) {
            v = far[i];
            const int32_t d = sssp_dist(key[v]);
            pk = d >= T1;
            pn = !pk && d >= T0;
            if (!pk) farflag[v] = 0;
        }
        const int64_t sn = block_append(nnear, pn, sc);
        if (pn) near[sn] = v;
        const int64_t sk = block_append(nfar2, pk, sc);
        if (pk) far2[sk] = v;
    }
}

__global__ void k_nf_seed_min(int64_t nf, const int32_t *F, const uint64_t *key, int64_t *out) {
    int64_t best = 0;
    for (int64_t i = gtid(); i < nf; i += gstride()) {
        const int32_t d = sssp_dist(key[F[i]]);
        if (d < INF) best = max(best, (int64_t)(INF - d));
    }
    best = wave_max_i32((int32_t)best);
    if (lane_id() == 0 && best > 0) atomicMax((unsigned long long *)out, (unsigned long long)best);
}

static int sssp_push_nearfar(dg_graph *g, uint64_t *key, int64_t nf, int32_t delta, dg_batch_stats *st) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const size_t cap = (size_t)g->n + 1;
    if (!ws.farflag.p || ws.farflag.cap < cap || ws.far_ctr >= INT32_MAX - 4) {
        DG_TRY(ws.farflag.ensure(cap));
        DG_TRY(fill_i32(ws.farflag.p, 0, (int64_t)cap, s));
        ws.far_ctr = 0;
    }
    DG_TRY(ws.far0.ensure(cap));
    DG_TRY(ws.far1.ensure(cap));
    const int32_t fst = ++ws.far_ctr;
    int32_t *A = ws.f0.p, *B = ws.f1.p, *far = ws.far0.p, *far2 = ws.far1.p;
    // first threshold: nearest seed + delta (every seed is relaxed in the first round)
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_nf_seed_min, dim3(grid_for(nf)), dim3(256), 0, s, nf, A, key, ws.dcnt + C_AUX2);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    if (ws.hcnt[C_AUX2] == 0) return DG_OK;
    int32_t T = (int32_t)std::min<int64_t>((int64_t)(INF - ws.hcnt[C_AUX2]) + delta, INF);
    int64_t nnear = nf, nfar = 0;
    int steps = 0;
    int64_t relaxed = 0, edges = 0;
    for (;;) {
        while (nnear > 0) {
            int32_t stv;
            DG_TRY(next_stamp(g, &stv));
            DG_TRY(counters_clear(g));
            RelaxOp op{key, ws.stamp.p, stv, B, ws.dcnt + C_F1};
            DG_TRY(launch_expand(s, with_tally(make_args(g, g->fwd, A, nnear), ws.dcnt + C_EDGES), op, 8192));
            hipLaunchKernelGGL(k_nf_split, dim3(4096), dim3(256), 0, s, ws.dcnt + C_F1, B, key, T, A,
                               ws.dcnt + C_F0, far + nfar, ws.dcnt + C_AUX1, ws.farflag.p, fst);
            DG_HIP(hipGetLastError());
            DG_TRY(counters_read(g));
            relaxed += nnear;
            edges += ws.hcnt[C_EDGES];
            nnear = ws.hcnt[C_F0];
            nfar += ws.hcnt[C_AUX1];
            ++steps;
        }
        if (nfar == 0) break;
        DG_TRY(counters_clear(g));
        hipLaunchKernelGGL(k_nf_min, dim3(grid_for(nfar)), dim3(256), 0, s, nfar, far, key, T, ws.dcnt + C_AUX2);
        DG_HIP(hipGetLastError());
        DG_TRY(counters_read(g));
        const int64_t best = ws.hcnt[C_AUX2];
        const int32_t T1 = best == 0 ? INF : (int32_t)std::min<int64_t>((int64_t)(INF - best) + delta, INF);
        DG_TRY(counters_clear(g));
        hipLaunchKernelGGL(k_nf_refill, dim3(grid_for(nfar)), dim3(256), 0, s, nfar, far, key, T, T1, A,
                           ws.dcnt + C_F0, far2, ws.dcnt + C_AUX1, ws.farflag.p);
        DG_HIP(hipGetLastError());
        DG_TRY(counters_read(g));
        nnear = ws.hcnt[C_F0];
        nfar = ws.hcnt[C_AUX1];
        std::swap(far, far2);
        T = T1;
        if (best == 0) break;  // the pile held only stale entries (now cleared)
    }
    if (st) {
        st->sssp_steps += steps;
        st->sssp_relaxed += relaxed;
        st->edges_traversed += edges;
    }
    return DG_OK;
}

// Push relaxation from frontier f0 (nf vertices) until no distance drops.
static int sssp_push(dg_graph *g, uint64_t *key, int64_t nf, dg_batch_stats *st) {
    if (g->cfg.sssp_delta > 0 && nf > 0) return sssp_push_nearfar(g, key, nf, g->cfg.sssp_delta, st);
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    int32_t *F = ws.f0.p, *N = ws.f1.p;
    int steps = 0;
    int64_t relaxed = 0, edges = 0;
    while (nf > 0) {
        int32_t stv;
        DG_TRY(next_stamp(g, &stv));
        DG_TRY(counters_clear(g));
        RelaxOp op{key, ws.stamp.p, stv, N, ws.dcnt + C_F1};
        DG_TRY(launch_expand(s, with_tally(make_args(g, g->fwd, F, nf), ws.dcnt + C_EDGES), op, 8192));
        DG_TRY(counters_read(g));
        relaxed += nf;
        edges += ws.hcnt[C_EDGES];
        nf = ws.hcnt[C_F1];
        std::swap(F, N);
        ++steps;
    }
    if (st) {
        st->sssp_steps += steps;
        st->sssp_relaxed += relaxed;
        st->edges_traversed += edges;
    }
    return DG_OK;
}

__global__ void k_sssp_set_sources(const int32_t *src, int64_t ns, uint64_t *key) {
    for (int64_t i = gtid(); i < ns; i += gstride()) key[src[i]] = sssp_pack(0, -1);
}

// ---- guard of the work-queue schedule --------------------------------------------------
// The work queue relaxes in FIFO order.  On a graph whose shortest-path trees are
// many hops deep and whose weights vary (a road network, a grid), FIFO order
// improves a vertex about once per wave of improvements that sweeps past it, so the
// work grows with the hop depth (a CPU model of a 4096 x 4096 grid improved every
// vertex hundreds of times).  Before the queue runs a static solve, a breadth-first
// probe from the sources counts hop levels; past WL_MAX_DEPTH levels the graph is
// refused, and the frontier schedules (near-far buckets for such graphs) remain.
constexpr int WL_MAX_DEPTH = 64;

struct DepthOp {
    int32_t *stamp;
    int32_t st;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t, int32_t &pay) const { pay = 0; return true; }
    __device__ bool edge(bool valid, int32_t, int32_t, int32_t x, int32_t) const {
        return valid && stamp[x] != st && atomicExch(&stamp[x], st) != st;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

__global__ void k_stamp_all(const int32_t *a, int64_t n, int32_t *stamp, int32_t st) {
    for (int64_t i = gtid(); i < n; i += gstride()) stamp[a[i]] = st;
}

// Hop levels of a breadth-first search from the ns sources in srcs, up to
// `limit` levels: *deep = true when vertices are still being discovered after it.
// The levels alternate between the near-far pile buffers (idle during a static
// solve), so srcs -- which may be the frontier buffer f0 -- is only read.
static int hop_depth_exceeds(dg_graph *g, const int32_t *srcs, int64_t ns, int limit, bool *deep) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const size_t cap = (size_t)g->n + 1;
    DG_TRY(ws.far0.ensure(cap));
    DG_TRY(ws.far1.ensure(cap));
    int32_t st;
    DG_TRY(next_stamp(g, &st));
    hipLaunchKernelGGL(k_stamp_all, dim3(grid_for(ns)), dim3(256), 0, s, srcs, ns, ws.stamp.p, st);
    DG_HIP(hipGetLastError());
    DG_HIP(hipMemcpyAsync(ws.far0.p, srcs, (size_t)ns * 4, hipMemcpyDeviceToDevice, s));
    int32_t *F = ws.far0.p, *N = ws.far1.p;
    int64_t nf = ns;
    int level = 0;
    while (nf > 0 && level < limit) {
        DG_TRY(counters_clear(g));
        DepthOp op{ws.stamp.p, st, N, ws.dcnt + C_F1};
        DG_TRY(launch_expand(s, make_args(g, g->fwd, F, nf), op, 8192));
        DG_TRY(counters_read(g));
        nf = ws.hcnt[C_F1];
        std::swap(F, N);
        ++level;
    }
    *deep = nf > 0;
    return DG_OK;
}

// Static solve from ns distinct sources (device array) -- one per member graph
// of a batched set, or a single source.
int sssp_static_multi(dg_graph *g, uint64_t *key, const int32_t *srcs, int64_t ns, dg_batch_stats *st) {
    hipStream_t s = g->stream;
    DG_TRY(ensure_frontiers(g));
    hipLaunchKernelGGL(k_sssp_init, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, key, -1);
    hipLaunchKernelGGL(k_sssp_set_sources, dim3(grid_for(ns)), dim3(256), 0, s, srcs, ns, key);
    DG_HIP(hipGetLastError());
    if (g->cfg.sssp_persistent == 1) {
        bool deep = false;
        DG_TRY(hop_depth_exceeds(g, srcs, ns, WL_MAX_DEPTH, &deep));
        if (deep)
            return set_error(DG_EINVAL, "work-queue schedule refused: shortest-path trees deeper than %d hops "
                                        "(FIFO relaxation would repeat work on such a graph); use "
                                        "sssp_persistent 0 or 2, with sssp_delta > 0 for road-like graphs",
                             WL_MAX_DEPTH);
        DG_TRY(sssp_static_persistent(g, key, srcs, ns));
        DG_HIP(hipStreamSynchronize(s));
        return DG_OK;
    }
    if (srcs != g->ws.f0.p)
        DG_HIP(hipMemcpyAsync(g->ws.f0.p, srcs, (size_t)ns * 4, hipMemcpyDeviceToDevice, s));
    DG_TRY(sssp_push(g, key, ns, st));
    return DG_OK;
}

int sssp_static_solve(dg_graph *g, uint64_t *key, int32_t source, dg_batch_stats *st) {
    DG_TRY(ensure_frontiers(g));
    int32_t src = source;
    DG_HIP(hipMemcpyAsync(g->ws.f0.p, &src, 4, hipMemcpyHostToDevice, g->stream));
    DG_HIP(hipStreamSynchronize(g->stream));
    return sssp_static_multi(g, key, g->ws.f0.p, 1, st);
}

int sssp_init(dg_query *q) {
    dg_graph *g = q->g;
    DG_TRY(q->key.ensure((size_t)g->n + 1));
    DG_TRY(q->inval.ensure((size_t)g->n + 1));
    q->nseeds = 0;
    if (q->nsrc > 0) return sssp_static_multi(g, q->key.p, q->srcs.p, q->nsrc, nullptr);
    return sssp_static_solve(g, q->key.p, q->source, nullptr);
}

int sssp_pre_delete(dg_query *q, int64_t adel) {
    dg_graph *g = q->g;
    q->nseeds = 0;
    if (adel <= 0) return DG_OK;
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_sssp_on_delete, dim3(grid_for(adel)), dim3(256), 0, g->stream, adel,
                       g->ws.adu.p, g->ws.adv.p, q->key.p, q->inval.p, g->ws.dcnt + C_AUX0);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    q->nseeds = g->ws.hcnt[C_AUX0];
    return DG_OK;
}

// ---- frontier rounds captured in hipGraphs ---------------------------------------------
// The same four steps as the host-driven path, with every count, frontier length,
// dedup stamp and (near-far) bucket threshold kept in device memory, so that a
// fixed number of frontier steps can be captured once into a hipGraph and replayed
// for every batch: the cut walk (CUT_LEVELS levels) in one graph, the pull, the
// seeding and PUSH_ROUNDS push rounds in another.  A step whose frontier is empty
// does nothing, so the graphs fit any batch.  Termination is decided on the device
// as well: each graph ends where a second graph, holding only the same rounds,
// continues from the device-resident counts (an even number of rounds per graph
// brings the frontier back to the buffer it started in), and the host replays that
// graph until the counts it reads after each replay are zero -- one host round
// trip per replay instead of one per step.  Kernel boundaries are the only
// grid-wide barriers, and no counter is contended beyond one append per wave.
enum {
    R_CA = 8, R_CB, R_LIST, R_PA, R_PB, R_STAMP, R_STEPS,
    // near-far rounds: relaxation output count, far-pile size and its other buffer's
    // count, which far buffer holds the pile, threshold T, smallest pile distance
    // (as INF - d), advance flag of the round, membership stamp of this batch
    R_NB, R_NF, R_NF2, R_FPAR, R_T, R_BEST, R_ADV, R_FST,
    R_EDGES,  // adjacency entries the steps examined (the traversal tally)
    R_END
};  // slots of q->qcnt
constexpr int CUT_LEVELS = 8, PUSH_ROUNDS = 16, NF_ROUNDS = 16;
static_assert(R_END <= 32, "round counters must fit the pinned staging block");
static_assert((CUT_LEVELS % 2) == 0 && (PUSH_ROUNDS % 2) == 0 && (NF_ROUNDS % 2) == 0,
              "a continuation graph must end in the buffer it starts from");
constexpr int HPIN_SLOTS = 32;

// Next step: zero the output count and the heavy-chunk count, advance the stamp,
// count the step if its input frontier is non-empty.
__global__ void k_round_prep(int64_t *out_cnt, int64_t *hcount, int64_t *ctr, const int64_t *in_cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (out_cnt) *out_cnt = 0;
        *hcount = 0;
        ctr[R_STAMP] += 1;
        if (in_cnt && *in_cnt > 0) ctr[R_STEPS] += 1;
    }
}

__global__ void k_rounds_init(int64_t *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[R_LIST] = ctr[0];  // the cut list starts with the pre-hook's seeds
        ctr[R_STEPS] = 0;
        ctr[R_EDGES] = 0;
    }
}

// Cut walk that also appends every cut vertex to the cut list.
struct CutListOp {
    uint64_t *key;
    int32_t *next;
    int64_t *ncount;
    int32_t *list;
    int64_t *lcount;
    __device__ bool vtx(int32_t, int32_t &pay) const { pay = 0; return true; }
    __device__ bool edge(bool valid, int32_t v, int32_t, int32_t x, int32_t) const {
        bool cut = false;
        if (valid) {
            uint64_t k = key[x];
            if (sssp_parent(k) == v) {
                key[x] = sssp_pack(INF, -1);
                cut = true;
            }
        }
        return cut;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount, list, lcount}; }
};

// RelaxOp with the round's stamp read from device memory.
struct RelaxOpD {
    uint64_t *key;
    int32_t *stamp;
    const int64_t *stp;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t v, int32_t &pay) const {
        int32_t d = sssp_dist(__atomic_load_n(&key[v], __ATOMIC_RELAXED));
        pay = d;
        return d < INF;
    }
    __device__ bool edge(bool valid, int32_t v, int32_t d, int32_t x, int32_t w) const {
        bool push = false;
        if (valid) {
            uint64_t cand = sssp_pack(d + w, v);
            if (cand < __atomic_load_n(&key[x], __ATOMIC_RELAXED)) {
                uint64_t old = atomicMin((unsigned long long *)&key[x], (unsigned long long)cand);
                if (cand < old && sssp_dist(cand) < sssp_dist(old)) {
                    const int32_t st = (int32_t)*stp;
                    push = atomicExch(&stamp[x], st) != st;
                }
            }
        }
        return push;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

__global__ void k_sssp_pulled_d(const int64_t *nc_p, const int32_t *cut, const uint64_t *key, int32_t *stamp,
                                const int64_t *stp, int32_t *front, int64_t *count) {
    __shared__ BlockScratch sc;
    const int64_t nc = *nc_p;
    const int32_t st = (int32_t)*stp;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < nc) {
            v = cut[i];
            p = sssp_dist(key[v]) < INF && atomicExch(&stamp[v], st) != st;
        }
        int64_t slot = block_append(count, p, sc);
        if (p) front[slot] = v;
    }
}

__global__ void k_sssp_on_add_d(const int64_t *na_p, const int32_t *aiu, const int32_t *aiv, const int32_t *aiw,
                                uint64_t *key, int32_t *stamp, const int64_t *stp, int32_t *front, int64_t *count) {
    __shared__ BlockScratch sc;
    const int64_t na = *na_p;
    const int32_t st = (int32_t)*stp;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < na) {
            int32_t u = aiu[i];
            v = aiv[i];
            int32_t du = sssp_dist(key[u]);
            if (du < INF) {
                uint64_t cand = sssp_pack(du + aiw[i], u);
                uint64_t old = atomicMin((unsigned long long *)&key[v], (unsigned long long)cand);
                if (cand < old && sssp_dist(cand) < sssp_dist(old)) p = atomicExch(&stamp[v], st) != st;
            }
        }
        int64_t slot = block_append(count, p, sc);
        if (p) front[slot] = v;
    }
}

// ---- near-far rounds with device-side state --------------------------------------------
// The near-far schedule of sssp_push_nearfar with its threshold, pile size, pile
// buffer and membership stamp in q->qcnt.  A round relaxes the near frontier into
// an output list, splits that list into the next near frontier (dist < T) and the
// far pile, and, when the near frontier came out empty while the pile is not,
// advances the bucket: T1 = (smallest pile distance >= T) + delta, entries in
// [T, T1) become the near frontier, entries >= T1 stay, stale ones leave.  Every
// kernel reads the counts and T from device memory and does nothing when its work
// is empty, so the rounds can be captured and replayed.

// Reset for a batch: empty pile, fresh membership stamp.
__global__ void k_nfd_reset(int64_t *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[R_BEST] = 0;
        ctr[R_NF] = 0;
        ctr[R_NF2] = 0;
        ctr[R_FPAR] = 0;
        ctr[R_ADV] = 0;
        ctr[R_FST] += 1;
    }
}

// Smallest finite distance of the seeds, as INF - d through a max (0: none).
__global__ void k_nfd_seed_min(const int64_t *nf_p, const int32_t *F, const uint64_t *key, int64_t *out) {
    const int64_t nf = *nf_p;
    int64_t best = 0;
    for (int64_t i = gtid(); i < nf; i += gstride()) {
        const int32_t d = sssp_dist(key[F[i]]);
        if (d < INF) best = max(best, (int64_t)(INF - d));
    }
    best = wave_max_i32((int32_t)best);
    if (lane_id() == 0 && best > 0) atomicMax((unsigned long long *)out, (unsigned long long)best);
}

// First threshold: nearest seed + delta (INF when no seed is finite: nothing moves).
__global__ void k_nfd_start(int64_t *ctr, int32_t delta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t best = ctr[R_BEST];
        ctr[R_T] = best == 0 ? (int64_t)INF : min((int64_t)(INF - best) + delta, (int64_t)INF);
    }
}

__device__ __forceinline__ int32_t nfd_next_threshold(int64_t best, int32_t delta) {
    return best == 0 ? INF : (int32_t)min((int64_t)(INF - best) + delta, (int64_t)INF);
}

// The previous round's bucket advance takes effect (when it advanced: the kept
// entries are the pile, T moves to T1), then this round's set-up: zero the
// relaxation, near-output, heavy-chunk and advance counts, advance the dedup stamp,
// count the step if its near frontier is non-empty.  in_cnt == nullptr: commit only.
__global__ void k_nfd_step(int64_t *ctr, int32_t delta, const int64_t *in_cnt, int64_t *out_cnt, int64_t *hcount) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ctr[R_ADV] != 0) {
        ctr[R_T] = nfd_next_threshold(ctr[R_BEST], delta);
        ctr[R_NF] = ctr[R_NF2];
        ctr[R_FPAR] ^= 1;
        ctr[R_ADV] = 0;
    }
    if (!in_cnt) return;
    *out_cnt = 0;
    *hcount = 0;
    ctr[R_NB] = 0;
    ctr[R_BEST] = 0;
    ctr[R_NF2] = 0;
    ctr[R_STAMP] += 1;
    if (*in_cnt > 0) ctr[R_STEPS] += 1;
}

// Relaxed vertices (count at ctr[R_NB]) -> next near frontier (dist < T) or the pile.
__global__ void k_nfd_split(const int32_t *N, const uint64_t *key, int64_t *ctr, int32_t *near, int64_t *nnear,
                            int32_t *far0, int32_t *far1, int32_t *farflag) {
    __shared__ BlockScratch sc;
    const int64_t nn = ctr[R_NB];
    const int32_t T = (int32_t)ctr[R_T], fst = (int32_t)ctr[R_FST];
    int32_t *far = ctr[R_FPAR] ? far1 : far0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nn; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        bool pn = false, pf = false;
        int32_t v = 0;
        if (i < nn) {
            v = N[i];
            pn = sssp_dist(key[v]) < T;
            pf = !pn && atomicExch(&farflag[v], fst) != fst;
        }
        const int64_t sn = block_append(nnear, pn, sc);
        if (pn) near[sn] = v;
        const int64_t sf = block_append(ctr + R_NF, pf, sc);
        if (pf) far[sf] = v;
    }
}

// The round advances the bucket when its near output is empty and the pile is
// not (the split is done, so the near count is final here; the refill that appends
// to it reads the decision from R_ADV).  Then: smallest pile distance >= T, as
// INF - d through a max (0: none).
__global__ void k_nfd_min(int64_t *ctr, const int64_t *nnear, const int32_t *far0, const int32_t *far1,
                          const uint64_t *key) {
    const bool adv = *nnear == 0 && ctr[R_NF] > 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[R_ADV] = adv ? 1 : 0;
    if (!adv) return;
    const int64_t nf = ctr[R_NF];
    const int32_t T = (int32_t)ctr[R_T];
    const int32_t *far = ctr[R_FPAR] ? far1 : far0;
    int64_t best = 0;
    for (int64_t i = gtid(); i < nf; i += gstride()) {
        const int32_t d = sssp_dist(key[far[i]]);
        if (d >= T && d < INF) best = max(best, (int64_t)(INF - d));
    }
    best = wave_max_i32((int32_t)best);
    if (lane_id() == 0 && best > 0) atomicMax((unsigned long long *)(ctr + R_BEST), (unsigned long long)best);
}

// Next bucket: pile entries in [T, T1) go near, entries >= T1 stay (other buffer),
// the rest are stale; entries leaving the pile clear their membership stamp.
__global__ void k_nfd_refill(int64_t *ctr, int32_t *far0, int32_t *far1, const uint64_t *key, int32_t delta,
                             int32_t *near, int64_t *nnear, int32_t *farflag) {
    __shared__ BlockScratch sc;
    if (ctr[R_ADV] == 0) return;
    const int64_t nf = ctr[R_NF];
    const int32_t T0 = (int32_t)ctr[R_T], T1 = nfd_next_threshold(ctr[R_BEST], delta);
    const int32_t *far = ctr[R_FPAR] ? far1 : far0;
    int32_t *far2 = ctr[R_FPAR] ? far0 : far1;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        bool pn = false, pk = false;
        int32_t v = 0;
        if (i < nf) {
            v = far[i];
            const int32_t d = sssp_dist(key[v]);
            pk = d >= T1;
            pn = !pk && d >= T0;
            if (!pk) farflag[v] = 0;
        }
        const int64_t sn = block_append(nnear, pn, sc);
        if (pn) near[sn] = v;
        const int64_t sk = block_append(ctr + R_NF2, pk, sc);
        if (pk) far2[sk] = v;
    }
}

static ExpandArgs dev_args(dg_graph *g, const Dir &d, const int32_t *F, const int64_t *nfp) {
    ExpandArgs a = make_args(g, d, F, 0);
    a.nfp = nfp;
    // captured rounds are replayed for later batches, when rows may have grown:
    // they keep the chunk kernel
    a.heavy_deg = heavy_deg(g);
    return a;
}

// Cut level: frontier F (count at *cf) -> N (count at *cn), cut list appended.
static int cut_level(dg_query *q, const int32_t *F, const int64_t *cf, int32_t *N, int64_t *cn) {
    dg_graph *g = q->g;
    int64_t *ctr = q->qcnt.p;
    hipLaunchKernelGGL(k_round_prep, dim3(1), dim3(64), 0, g->stream, cn, g->ws.dcnt + C_HEAVY, ctr, nullptr);
    CutListOp op{q->key.p, N, cn, q->inval.p, ctr + R_LIST};
    DG_TRY(launch_expand(g->stream, with_tally(dev_args(g, g->fwd, F, cf), ctr + R_EDGES), op, 1024));
    return DG_OK;
}

// Push round: frontier F (count at *cf) -> N (count at *cn).
static int push_round(dg_query *q, const int32_t *F, const int64_t *cf, int32_t *N, int64_t *cn) {
    dg_graph *g = q->g;
    int64_t *ctr = q->qcnt.p;
    hipLaunchKernelGGL(k_round_prep, dim3(1), dim3(64), 0, g->stream, cn, g->ws.dcnt + C_HEAVY, ctr, cf);
    RelaxOpD op{q->key.p, q->gstamp.p, ctr + R_STAMP, N, cn};
    DG_TRY(launch_expand(g->stream, with_tally(dev_args(g, g->fwd, F, cf), ctr + R_EDGES), op, 1024));
    return DG_OK;
}

// Cut levels alternate f0 (count R_CA) and f1 (R_CB).  first: level 0 walks the
// seeds (the head of the cut list) into f0; otherwise the levels continue from f1,
// where the previous graph's last level left its output.
static int rounds_cut_enqueue(dg_query *q, bool first) {
    dg_graph *g = q->g;
    int64_t *ctr = q->qcnt.p;
    int l0 = 0;
    if (first) {
        hipLaunchKernelGGL(k_rounds_init, dim3(1), dim3(64), 0, g->stream, ctr);
        DG_TRY(cut_level(q, q->inval.p, ctr + 0, g->ws.f0.p, ctr + R_CA));
        l0 = 1;
    }
    for (int l = l0; l < CUT_LEVELS; ++l) {
        const bool from_a = (l & 1) != 0;  // odd levels read f0, even levels f1
        DG_TRY(cut_level(q, from_a ? g->ws.f0.p : g->ws.f1.p, ctr + (from_a ? R_CA : R_CB),
                         from_a ? g->ws.f1.p : g->ws.f0.p, ctr + (from_a ? R_CB : R_CA)));
    }
    DG_HIP(hipGetLastError());
    return DG_OK;
}

// Near-far round: near frontier F (count *cf) -> relaxed list nfout (R_NB) -> next
// near frontier N (count *cn) and the pile; then the bucket advance if N is empty
// (taking effect in the next round's set-up, or the graph's closing commit).  The
// kernels that only act on an advance run on small grids: most rounds skip them.
static int nf_round(dg_query *q, const int32_t *F, const int64_t *cf, int32_t *N, int64_t *cn) {
    dg_graph *g = q->g;
    Work &ws = g->ws;
    hipStream_t s = g->stream;
    int64_t *ctr = q->qcnt.p;
    const int32_t delta = g->cfg.sssp_delta;
    hipLaunchKernelGGL(k_nfd_step, dim3(1), dim3(64), 0, s, ctr, delta, cf, cn, ws.dcnt + C_HEAVY);
    RelaxOpD op{q->key.p, q->gstamp.p, ctr + R_STAMP, ws.nfout.p, ctr + R_NB};
    DG_TRY(launch_expand(s, with_tally(dev_args(g, g->fwd, F, cf), ctr + R_EDGES), op, 1024));
    hipLaunchKernelGGL(k_nfd_split, dim3(256), dim3(256), 0, s, ws.nfout.p, q->key.p, ctr, N, cn, ws.far0.p,
                       ws.far1.p, q->gfar.p);
    hipLaunchKernelGGL(k_nfd_min, dim3(64), dim3(256), 0, s, ctr, cn, ws.far0.p, ws.far1.p, q->key.p);
    hipLaunchKernelGGL(k_nfd_refill, dim3(64), dim3(256), 0, s, ctr, ws.far0.p, ws.far1.p, q->key.p, delta, N, cn,
                       q->gfar.p);
    return DG_OK;
}

// Push rounds alternate f0 (count R_PA) and f1 (R_PB) and end in f0.  first: the
// pull at every cut vertex and the seeding come first (and, near-far, the bucket
// set-up).  Near-far rounds when sssp_delta > 0.
static int rounds_push_enqueue(dg_query *q, bool first) {
    dg_graph *g = q->g;
    Work &ws = g->ws;
    hipStream_t s = g->stream;
    int64_t *ctr = q->qcnt.p;
    const bool nf = g->cfg.sssp_delta > 0;
    if (first) {
        // pull once at every cut vertex
        hipLaunchKernelGGL(k_round_prep, dim3(1), dim3(64), 0, s, nullptr, ws.dcnt + C_HEAVY, ctr, nullptr);
        DG_TRY(launch_expand(s, with_tally(dev_args(g, *g->rev, q->inval.p, ctr + R_LIST), ctr + R_EDGES),
                             PullOp{q->key.p}, 1024));
        // seeds: pulled cut vertices and improved heads of inserted arcs
        hipLaunchKernelGGL(k_round_prep, dim3(1), dim3(64), 0, s, ctr + R_PA, ws.dcnt + C_HEAVY, ctr, nullptr);
        hipLaunchKernelGGL(k_sssp_pulled_d, dim3(1024), dim3(256), 0, s, ctr + R_LIST, q->inval.p, q->key.p,
                           q->gstamp.p, ctr + R_STAMP, ws.f0.p, ctr + R_PA);
        hipLaunchKernelGGL(k_sssp_on_add_d, dim3(1024), dim3(256), 0, s, ctr + 1, ws.aiu.p, ws.aiv.p, ws.aiw.p,
                           q->key.p, q->gstamp.p, ctr + R_STAMP, ws.f0.p, ctr + R_PA);
        if (nf) {
            hipLaunchKernelGGL(k_nfd_reset, dim3(1), dim3(64), 0, s, ctr);
            hipLaunchKernelGGL(k_nfd_seed_min, dim3(1024), dim3(256), 0, s, ctr + R_PA, ws.f0.p, q->key.p,
                               ctr + R_BEST);
            hipLaunchKernelGGL(k_nfd_start, dim3(1), dim3(64), 0, s, ctr, g->cfg.sssp_delta);
        }
    }
    const int rounds = nf ? NF_ROUNDS : PUSH_ROUNDS;
    for (int r = 0; r < rounds; ++r) {
        const bool even = (r & 1) == 0;
        const int32_t *F = even ? ws.f0.p : ws.f1.p;
        int32_t *N = even ? ws.f1.p : ws.f0.p;
        const int64_t *cf = ctr + (even ? R_PA : R_PB);
        int64_t *cn = ctr + (even ? R_PB : R_PA);
        if (nf) DG_TRY(nf_round(q, F, cf, N, cn));
        else DG_TRY(push_round(q, F, cf, N, cn));
    }
    // the last round's advance takes effect before the host reads the counts
    if (nf)
        hipLaunchKernelGGL(k_nfd_step, dim3(1), dim3(64), 0, s, ctr, g->cfg.sssp_delta, (const int64_t *)nullptr,
                           (int64_t *)nullptr, (int64_t *)nullptr);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

static int rounds_read(dg_query *q, int64_t *h) {
    dg_graph *g = q->g;
    DG_HIP(hipMemcpyAsync(q->hpin, q->qcnt.p, R_END * sizeof(int64_t), hipMemcpyDeviceToHost, g->stream));
    DG_HIP(wait_stream(g, g->stream));
    std::memcpy(h, q->hpin, R_END * sizeof(int64_t));
    return DG_OK;
}

static int sssp_post_rounds(dg_query *q, int64_t ains, dg_batch_stats *st) {
    dg_graph *g = q->g;
    Work &ws = g->ws;
    const bool nf = g->cfg.sssp_delta > 0;
    DG_TRY(ensure_frontiers(g));
    if (!q->hpin) DG_HIP(hipHostMalloc((void **)&q->hpin, HPIN_SLOTS * sizeof(int64_t), hipHostMallocDefault));
    if (!q->gstamp.p || q->gstamp.cap < (size_t)g->n + 1 || q->qcnt.cap < (size_t)R_END) {
        // stamps and their counters start together (a stamp is never reused)
        DG_TRY(q->qcnt.ensure(R_END, true, g->stream));
        DG_TRY(q->gstamp.ensure((size_t)g->n + 1));
        DG_TRY(fill_i32(q->gstamp.p, 0, g->n + 1, g->stream));
        DG_TRY(fill_i64(q->qcnt.p, 0, R_END, g->stream));
    }
    if (nf) {
        const size_t cap = (size_t)g->n + 1;
        DG_TRY(ws.far0.ensure(cap));
        DG_TRY(ws.far1.ensure(cap));
        DG_TRY(ws.nfout.ensure(cap));
        if (!q->gfar.p || q->gfar.cap < cap) {
            // membership stamps and their counter start together
            DG_TRY(q->gfar.ensure(cap));
            DG_TRY(fill_i32(q->gfar.p, 0, (int64_t)cap, g->stream));
            DG_TRY(fill_i64(q->qcnt.p + R_FST, 0, 1, g->stream));
        }
    }
    if (!q->gcache) {
        q->own_cache = new GraphCache();
        q->gcache = q->own_cache;
    }
    q->hpin[0] = q->nseeds;
    q->hpin[1] = ains;
    DG_HIP(hipMemcpyAsync(q->qcnt.p, q->hpin, 2 * sizeof(int64_t), hipMemcpyHostToDevice, g->stream));
    const Dir &R = *g->rev;
    std::vector<const void *> sig = {q->key.p, q->inval.p, q->qcnt.p, q->gstamp.p, ws.f0.p, ws.f1.p, ws.heavy.p,
                                     ws.dcnt, g->fwd.off.p, g->fwd.col.p, g->fwd.w.p, g->fwd.doff.p,
                                     g->fwd.dcol.p, g->fwd.dw.p, R.off.p, R.col.p, R.w.p, R.doff.p, R.dcol.p, R.dw.p,
                                     ws.aiu.p, ws.aiv.p, ws.aiw.p,
                                     reinterpret_cast<const void *>((intptr_t)heavy_deg(g))};
    if (nf) {
        sig.push_back(ws.far0.p);
        sig.push_back(ws.far1.p);
        sig.push_back(ws.nfout.p);
        sig.push_back(q->gfar.p);
        sig.push_back(reinterpret_cast<const void *>((intptr_t)g->cfg.sssp_delta));
    }
    int64_t h[R_END];
    // the legacy null stream cannot be captured: launch the same steps directly
    auto run = [&](const char *tag, const std::function<int()> &enqueue) {
        if (!g->stream) return enqueue();
        sig.push_back(tag);
        const int rc = graph_replay(g, q->gcache, sig, enqueue);
        sig.pop_back();
        return rc;
    };
    // 1. cut walk: the first graph, then its continuation until the last level's
    //    output (f1) is empty
    // Bellman-Ford settles within n rounds and a cut walk within n levels: a replay
    // count far beyond that means the device state is inconsistent, not slow work
    const int64_t max_replays = 4 * ((int64_t)g->n / std::min(CUT_LEVELS, PUSH_ROUNDS) + 1) + 1024;
    int64_t replays = 0;
    DG_TRY(run("cut", [&]() { return rounds_cut_enqueue(q, true); }));
    DG_TRY(rounds_read(q, h));
    while (h[R_CB] > 0) {
        if (++replays > max_replays) return set_error(DG_EDEVICE, "SSSP cut walk did not terminate (internal error)");
        DG_TRY(run("cut+", [&]() { return rounds_cut_enqueue(q, false); }));
        DG_TRY(rounds_read(q, h));
    }
    const int64_t ncut = h[R_LIST];
    // 2-4. pull, seeds, push (or near-far) rounds, continued until the frontier
    //      (and the far pile) are empty
    DG_TRY(run(nf ? "nf" : "push", [&]() { return rounds_push_enqueue(q, true); }));
    DG_TRY(rounds_read(q, h));
    while (h[R_PA] > 0 || (nf && h[R_NF] > 0)) {
        if (++replays > max_replays)
            return set_error(DG_EDEVICE, "SSSP push rounds did not terminate (internal error)");
        DG_TRY(run(nf ? "nf+" : "push+", [&]() { return rounds_push_enqueue(q, false); }));
        DG_TRY(rounds_read(q, h));
    }
    if (st) {
        st->sssp_invalidated += ncut;
        st->sssp_steps += (int32_t)h[R_STEPS];
        st->edges_traversed += h[R_EDGES];
    }
    return DG_OK;
}

int sssp_post_update(dg_query *q, int64_t adel, int64_t ains, dg_batch_stats *st) {
    (void)adel;
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    DG_TRY(ensure_frontiers(g));
    // 2: frontier rounds with device-side counts and termination, captured and
    // replayed.  The default (0, as 3) launches each step from the host with a grid
    // sized to its frontier and reads its count: measured faster on this GPU, where
    // a replayed graph node costs more than the round trip it saves (SSSP alone, 100k
    // batches: R-MAT 22 about equal, 4096^2 grid with near-far buckets 15-23 ms per
    // batch host-driven against 21-32 ms captured; beside the PageRank steps the
    // fixed grid-stride grids of the captured rounds also slowed the tile kernel).
    if (g->cfg.sssp_persistent == 2) return sssp_post_rounds(q, ains, st);
    if (g->cfg.sssp_persistent == 1) {
        // the same four steps on device work queues, without host round trips
        DG_TRY(q->qcnt.ensure(4));
        if (!q->hpin) DG_HIP(hipHostMalloc((void **)&q->hpin, HPIN_SLOTS * sizeof(int64_t), hipHostMallocDefault));
        q->hpin[0] = q->nseeds;
        q->hpin[1] = ains;
        DG_HIP(hipMemcpyAsync(q->qcnt.p, q->hpin, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
        int64_t ncut = 0, edges = 0;
        if (q->gcache)
            DG_TRY(sssp_post_graph(g, q->gcache, q->key.p, q->inval.p, q->qcnt.p, ws.f1.p, q->qcnt.p + 1, &ncut,
                                   &edges));
        else
            DG_TRY(sssp_post_persistent(g, q->key.p, q->inval.p, q->qcnt.p, ws.f1.p, q->qcnt.p + 1, &ncut,
                                        &edges));
        if (st) {
            st->sssp_invalidated += ncut;
            st->sssp_steps += 1;
            st->edges_traversed += edges;
        }
        return DG_OK;
    }
    // 1. cut the subtrees below the seeds; q->inval collects every cut vertex
    int64_t ncut = q->nseeds;
    int64_t lo = 0, hi = ncut, edges = 0;
    while (hi > lo) {
        DG_TRY(counters_clear(g));
        CutOp op{q->key.p, q->inval.p + hi, ws.dcnt + C_F1};
        DG_TRY(launch_expand(s, with_tally(make_args(g, g->fwd, q->inval.p + lo, hi - lo), ws.dcnt + C_EDGES), op,
                             8192));
        DG_TRY(counters_read(g));
        edges += ws.hcnt[C_EDGES];
        lo = hi;
        hi += ws.hcnt[C_F1];
    }
    ncut = hi;
    if (st) st->sssp_invalidated += ncut;
    // 2. one pull per cut vertex over its live in-edges
    DG_TRY(counters_clear(g));
    if (ncut > 0) {
        PullOp op{q->key.p};
        DG_TRY(launch_expand(s, with_tally(make_args(g, *g->rev, q->inval.p, ncut), ws.dcnt + C_EDGES), op, 8192));
    }
    // 3. inserted arcs relax their heads; 2+3 seed the push frontier
    int32_t stv;
    DG_TRY(next_stamp(g, &stv));
    if (ncut > 0)
        hipLaunchKernelGGL(k_sssp_pulled, dim3(grid_for(ncut)), dim3(256), 0, s, ncut, q->inval.p,
                           q->key.p, ws.stamp.p, stv, ws.f0.p, ws.dcnt + C_F0);
    if (ains > 0)
        hipLaunchKernelGGL(k_sssp_on_add, dim3(grid_for(ains)), dim3(256), 0, s, ains, ws.aiu.p,
                           ws.aiv.p, ws.aiw.p, q->key.p, ws.stamp.p, stv, ws.f0.p, ws.dcnt + C_F0);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    edges += ws.hcnt[C_EDGES];  // the pull's entries
    if (st) st->edges_traversed += edges;
    // 4. push to the fixed point
    return sssp_push(g, q->key.p, ws.hcnt[C_F0], st);
}

int sssp_unpack(dg_graph *g, const uint64_t *key, int32_t *dist, int32_t *parent, hipStream_t s) {
    const bool r = g->relabeled;
    hipLaunchKernelGGL(k_sssp_unpack, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, key,
                       r ? (const int32_t *)g->perm.p : nullptr, r ? (const int32_t *)g->iperm.p : nullptr, dist,
                       parent);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

// ---- checkpoint / resume -----------------------------------------------------------------
// A resumed query must hold the shortest-path solution of the graph it is attached
// to, since the dynamic update only repairs what a batch disturbs.  So an imported
// (dist, parent) pair is packed into keys and then checked against the current
// graph in one pass over its in-rows, which is much cheaper than a static solve:
//   - the source has (0, -1);
//   - no live arc u -> v with d[u] + w < INF improves on d[v] (optimality);
//   - every other vertex with d[v] < INF has a live in-arc from parent[v] with
//     d[parent] + w == d[v] (a tight tree arc), and every vertex with d[v] == INF
//     has parent -1.
// With positive weights the tight parent arcs strictly decrease d, so they form
// a tree rooted at the source, and the pair is exactly the saturated static result.

// dist/parent in the caller's ids -> keys in internal ids; *bad counts values
// outside [0, INF] or parents outside [-1, n).
__global__ void k_sssp_pack(int32_t n, const int32_t *dist, const int32_t *parent, const int32_t *perm,
                            uint64_t *key, int64_t *bad) {
    int64_t nbad = 0;
    for (int64_t c = gtid(); c < n; c += gstride()) {
        const int32_t d = dist[c], p = parent[c];
        const bool ok = d >= 0 && d <= INF && p >= -1 && p < n;
        nbad += ok ? 0 : 1;
        const int32_t pi = ok && p >= 0 ? (perm ? perm[p] : p) : -1;
        key[perm ? perm[c] : c] = sssp_pack(ok ? d : INF, pi);
    }
    nbad = wave_sum(nbad);
    if (lane_id() == 0 && nbad) atomicAdd((unsigned long long *)bad, (unsigned long long)nbad);
}

// One wave per in-row v (grid-stride); *bad counts the rows that break a rule above.
__global__ __launch_bounds__(256) void k_sssp_verify(int32_t n, int32_t source, DirView r, const uint64_t *key,
                                                     int64_t *bad) {
    const int64_t nwaves = gstride() / WAVE;
    const int l = lane_id();
    int64_t nbad = 0;
    for (int64_t v = gtid() / WAVE; v < n; v += nwaves) {
        const uint64_t kv = key[v];
        const int64_t dv = sssp_dist(kv);
        const int32_t pv = sssp_parent(kv);
        bool improves = false, tight = false;
        auto check = [&](uint32_t c, int32_t w) {
            if (c & DEAD) return;
            const int32_t u = (int32_t)(c & ID_MASK);
            const int64_t du = sssp_dist(key[u]);
            if (du >= INF) return;
            const int64_t s = du + (int64_t)w;
            if (s < INF && s < dv) improves = true;
            if (u == pv && s == dv) tight = true;
        };
        for (int64_t e = r.off[v] + l; e < r.off[v + 1]; e += WAVE) check((uint32_t)r.col[e], r.w[e]);
        for (int64_t e = r.doff[v] + l; e < r.doff[v + 1]; e += WAVE) check((uint32_t)r.dcol[e], r.dw[e]);
        improves = ballot(improves) != 0;
        tight = ballot(tight) != 0;
        bool ok;
        if (v == source) ok = dv == 0 && pv == -1;
        else if (dv < INF) ok = !improves && pv >= 0 && tight;
        else ok = !improves && pv == -1;
        if (l == 0 && !ok) ++nbad;
    }
    if (l == 0 && nbad) atomicAdd((unsigned long long *)bad, (unsigned long long)nbad);
}

int sssp_import(dg_query *q, const int32_t *dist, const int32_t *parent) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    DG_TRY(q->key.ensure((size_t)g->n + 1));
    DG_TRY(q->inval.ensure((size_t)g->n + 1));
    q->nseeds = 0;
    DG_TRY(g->ws.rbuf.ensure((size_t)g->n + 1));
    int32_t *tmp = reinterpret_cast<int32_t *>(g->ws.rbuf.p);  // 2n + 2 int32
    DG_HIP(hipMemcpyAsync(tmp, dist, (size_t)g->n * 4, hipMemcpyHostToDevice, s));
    DG_HIP(hipMemcpyAsync(tmp + g->n, parent, (size_t)g->n * 4, hipMemcpyHostToDevice, s));
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_sssp_pack, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, tmp, tmp + g->n,
                       g->relabeled ? (const int32_t *)g->perm.p : nullptr, q->key.p, g->ws.dcnt + C_AUX0);
    hipLaunchKernelGGL(k_sssp_verify, dim3(grid_for((int64_t)g->n * WAVE)), dim3(256), 0, s, g->n, q->source,
                       view(*g->rev), q->key.p, g->ws.dcnt + C_AUX1);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    if (g->ws.hcnt[C_AUX0] != 0)
        return set_error(DG_EINVAL, "imported shortest paths: %lld values out of range",
                         (long long)g->ws.hcnt[C_AUX0]);
    if (g->ws.hcnt[C_AUX1] != 0)
        return set_error(DG_EINVAL, "imported shortest paths do not solve this graph from its source (%lld "
                                    "vertices break optimality or tree tightness)",
                         (long long)g->ws.hcnt[C_AUX1]);
    return DG_OK;
}

int sssp_read(dg_query *q, int32_t *dist, int32_t *parent, bool dev) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    if (dev) {
        DG_TRY(sssp_unpack(g, q->key.p, dist, parent, s));
    } else {
        DG_TRY(g->ws.rbuf.ensure((size_t)g->n + 1));
        int32_t *tmp = reinterpret_cast<int32_t *>(g->ws.rbuf.p);  // 2n + 2 int32
        DG_TRY(sssp_unpack(g, q->key.p, tmp, tmp + g->n, s));
        hipError_t e1 = hipMemcpyAsync(dist, tmp, (size_t)g->n * 4, hipMemcpyDeviceToHost, s);
        hipError_t e2 = parent ? hipMemcpyAsync(parent, tmp + g->n, (size_t)g->n * 4, hipMemcpyDeviceToHost, s)
                               : hipSuccess;
        hipError_t e3 = hipStreamSynchronize(s);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            return set_error(DG_EDEVICE, "sssp read copy failed");
        return DG_OK;
    }
    DG_HIP(hipStreamSynchronize(s));
    return DG_OK;
}

}  // namespace dg
