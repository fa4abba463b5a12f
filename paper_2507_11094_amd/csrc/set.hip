// Batched sets of independent graphs and the tile-shape autotuner.
//
// A set keeps its member graphs as ONE device-resident store (the disjoint union,
// vertex ids offset by per-member bases), so a batch for every member is one
// batch for the store and all members' shortest paths move together: the cut
// walk and the push run as frontier rounds captured once into hipGraphs and
// replayed for every batch (sssp.hip), or, on request (sssp_persistent = 1), as
// persistent work-queue kernels (worklist.hip).  Members never share an edge, so
// each member's result is exactly what it would be alone.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>
#include <vector>

#include "dg_device.h"

struct dg_set {
    int32_t count = 0;
    std::vector<int64_t> vbase;  // count + 1
    dg::DBuf<int64_t> dvbase;
    dg::DBuf<int64_t> doff;      // element offsets of the call being translated
    dg::DBuf<int32_t> ts, td, tw;
    dg::DBuf<uint8_t> top;
    dg::DBuf<int64_t> derr;
    dg_graph *g = nullptr;
    dg_query *q = nullptr;
    dg::GraphCache cache;
    hipStream_t stream = nullptr;
};

namespace dg {

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

// Member-local -> store ids.  off: element offsets per member (count + 1); an id
// outside its member's [0, n_i) raises *err.
// Members hold runs of consecutive entries, so one search per block finds the member
// of the block's first entry and each thread steps forward from it (members with no
// entries are stepped over).
__global__ __launch_bounds__(256) void k_set_translate(int64_t total, const int64_t *off, int32_t count,
                                                       const int64_t *vbase, const int32_t *s, const int32_t *d,
                                                       int32_t *os, int32_t *od, int64_t *err) {
    __shared__ int32_t s_mb;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < total; b0 += (int64_t)gridDim.x * blockDim.x) {
        if (threadIdx.x == 0) s_mb = row_of(off, 0, count - 1, b0);
        __syncthreads();
        int32_t mb = s_mb;
        __syncthreads();  // s_mb is written again in the next pass
        const int64_t i = b0 + threadIdx.x;
        if (i >= total) continue;
        while (mb + 1 < count && off[mb + 1] <= i) ++mb;
        const int64_t b = vbase[mb], nl = vbase[mb + 1] - b;
        const int32_t u = s[i], v = d[i];
        if (u < 0 || u >= nl || v < 0 || v >= nl) {
            atomicOr((unsigned long long *)err, 1ull);
            os[i] = (int32_t)b;
            od[i] = (int32_t)b;
        } else {
            os[i] = (int32_t)(b + u);
            od[i] = (int32_t)(b + v);
        }
    }
}

__global__ void k_set_unpack(int64_t nl, const uint64_t *key, int64_t base, int32_t *dist, int32_t *parent) {
    for (int64_t v = gtid(); v < nl; v += gstride()) {
        uint64_t k = key[base + v];
        int32_t d = sssp_dist(k);
        dist[v] = d >= INF ? INF : d;
        if (parent) {
            int32_t p = d >= INF ? -1 : sssp_parent(k);
            parent[v] = p < 0 ? -1 : (int32_t)(p - base);
        }
    }
}

template <class T>
static int stage_into(const T *p, int64_t n, bool dev, hipStream_t s, DBuf<T> &buf, const T **out) {
    if (!p || dev) {
        *out = p;
        return DG_OK;
    }
    DG_TRY(buf.ensure((size_t)n + 1));
    if (n > 0) DG_HIP(hipMemcpyAsync(buf.p, p, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
    *out = buf.p;
    return DG_OK;
}

// Translate (src, dst) of `total` elements grouped per member by `counts`.
static int set_translate(dg_set *S, const int64_t *counts, int64_t total, const int32_t *src, const int32_t *dst,
                         bool dev, const int32_t **os, const int32_t **od) {
    hipStream_t s = S->stream;
    std::vector<int64_t> off(S->count + 1, 0);
    for (int32_t i = 0; i < S->count; ++i) {
        if (counts[i] < 0) return set_error(DG_EINVAL, "negative count for member %d", i);
        off[i + 1] = off[i] + counts[i];
    }
    if (off[S->count] != total) return set_error(DG_EINVAL, "count mismatch");
    DG_TRY(S->doff.ensure(S->count + 1));
    DG_TRY(S->derr.ensure(2));
    DG_HIP(hipMemcpyAsync(S->doff.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DG_TRY(fill_i32(reinterpret_cast<int32_t *>(S->derr.p), 0, 4, s));
    DBuf<int32_t> hs, hd;
    const int32_t *ds = nullptr, *dd = nullptr;
    DG_TRY(stage_into(src, total, dev, s, hs, &ds));
    DG_TRY(stage_into(dst, total, dev, s, hd, &dd));
    DG_TRY(S->ts.ensure(total + 1));
    DG_TRY(S->td.ensure(total + 1));
    if (total > 0)
        hipLaunchKernelGGL(k_set_translate, dim3(grid_for(total)), dim3(256), 0, s, total, S->doff.p, S->count,
                           S->dvbase.p, ds, dd, S->ts.p, S->td.p, S->derr.p);
    DG_HIP(hipGetLastError());
    int64_t err = 0;
    DG_HIP(hipMemcpyAsync(&err, S->derr.p, sizeof(err), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    hs.release();
    hd.release();
    if (err) return set_error(DG_EINVAL, "a vertex id lies outside its member graph");
    *os = S->ts.p;
    *od = S->td.p;
    return DG_OK;
}

// ---- tuning ------------------------------------------------------------------------------

// Time `apply` under each candidate configuration on a snapshot of g, keep the
// fastest.  Each candidate runs twice from the snapshot (the first run may build
// a captured graph or grow buffers) and its second time counts.
static int tune(dg_graph *g, const std::function<int()> &apply, dg_config *best, double *best_ms) {
    dg_snapshot *snap = nullptr;
    DG_TRY(dg_snapshot_save(g, &snap));
    const dg_config base = g->cfg;
    std::vector<dg_config> cands;
    const int heavies[] = {32, 64, 128, 256, 512};
    const int groups_p[] = {256, 512, 1024, 2048};
    for (int h : heavies) {
        if (base.sssp_persistent == 1) {
            for (int gp : groups_p) {
                dg_config c = base;
                c.heavy_degree = h;
                c.persistent_groups = gp;
                cands.push_back(c);
            }
        } else {
            dg_config c = base;
            c.heavy_degree = h;
            cands.push_back(c);
        }
    }
    double bms = 1e300;
    dg_config bc = base;
    int rc = DG_OK;
    for (const dg_config &c : cands) {
        g->cfg = c;
        double ms = 0.0;
        for (int rep = 0; rep < 2 && rc == DG_OK; ++rep) {
            rc = dg_snapshot_restore(g, snap);
            if (rc != DG_OK) break;
            auto t0 = std::chrono::steady_clock::now();
            rc = apply();
            (void)hipStreamSynchronize(g->stream);
            ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (rc != DG_OK) break;
        if (ms < bms) {
            bms = ms;
            bc = c;
        }
    }
    int rc2 = dg_snapshot_restore(g, snap);
    dg_snapshot_free(snap);
    g->cfg = rc == DG_OK ? bc : base;
    if (rc != DG_OK) return rc;
    if (rc2 != DG_OK) return rc2;
    if (best) *best = bc;
    if (best_ms) *best_ms = bms;
    return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" {

int dg_set_create(int32_t count, const int32_t *n, const int64_t *m, const int32_t *src, const int32_t *dst,
                  const int32_t *w, uint32_t flags, const dg_config *cfg, dg_set **out) {
    if (!out || count <= 0 || !n || !m) return set_error(DG_EINVAL, "bad set arguments");
    *out = nullptr;
    if (flags & ~(DG_DEVICE_PTRS)) return set_error(DG_EINVAL, "unknown flags (sets are directed)");
    int64_t nv = 0, na = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (n[i] <= 0 || m[i] < 0) return set_error(DG_EINVAL, "member %d: bad sizes", i);
        nv += n[i];
        na += m[i];
    }
    if (nv > (1 << 30)) return set_error(DG_EINVAL, "a set holds at most 2^30 vertices in total");
    if (na > 0 && (!src || !dst)) return set_error(DG_EINVAL, "null edge arrays");
    dg_set *S = new dg_set();
    S->count = count;
    S->vbase.assign(count + 1, 0);
    for (int32_t i = 0; i < count; ++i) S->vbase[i + 1] = S->vbase[i] + n[i];
    int rc = DG_OK;
    if (hipStreamCreate(&S->stream) != hipSuccess) rc = set_error(DG_EDEVICE, "stream creation failed");
    if (rc == DG_OK) rc = S->dvbase.ensure(count + 1);
    if (rc == DG_OK && hipMemcpy(S->dvbase.p, S->vbase.data(), (count + 1) * sizeof(int64_t),
                                 hipMemcpyHostToDevice) != hipSuccess)
        rc = set_error(DG_EDEVICE, "copy failed");
    const int32_t *os = nullptr, *od = nullptr, *dw = nullptr;
    DBuf<int32_t> hw;
    if (rc == DG_OK) rc = set_translate(S, m, na, src, dst, (flags & DG_DEVICE_PTRS) != 0, &os, &od);
    if (rc == DG_OK) rc = stage_into(w, na, (flags & DG_DEVICE_PTRS) != 0, S->stream, hw, &dw);
    dg_config c{};
    if (cfg) c = *cfg;
    if (c.sssp_persistent != 1) c.sssp_persistent = 2;  // captured frontier rounds unless the queue is asked for
    if (rc == DG_OK) rc = graph_create_dev((int32_t)nv, na, os, od, dw, &c, S->stream, &S->g);
    hw.release();
    S->ts.release();
    S->td.release();
    if (rc != DG_OK) {
        if (S->stream) (void)hipStreamDestroy(S->stream);
        S->dvbase.release();
        S->doff.release();
        S->derr.release();
        delete S;
        return rc;
    }
    *out = S;
    return DG_OK;
}

int dg_set_destroy(dg_set *S) {
    if (!S) return set_error(DG_EINVAL, "null set");
    graph_cache_clear(&S->cache);
    if (S->g) dg_graph_destroy(S->g);
    S->dvbase.release(); S->doff.release(); S->ts.release(); S->td.release(); S->tw.release();
    S->top.release(); S->derr.release();
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return DG_OK;
}

int dg_set_info(dg_set *S, int32_t *count, int64_t *vertices, int64_t *arcs) {
    if (!S) return set_error(DG_EINVAL, "null set");
    if (count) *count = S->count;
    if (vertices) *vertices = S->vbase[S->count];
    if (arcs) *arcs = S->g->m_live;
    return DG_OK;
}

int dg_set_sssp_attach(dg_set *S, const int32_t *sources) {
    if (!S || !sources) return set_error(DG_EINVAL, "bad arguments");
    if (S->q) return set_error(DG_ESTATE, "the set already has a shortest-path query");
    std::vector<int32_t> gs(S->count);
    for (int32_t i = 0; i < S->count; ++i) {
        if (sources[i] < 0 || sources[i] >= S->vbase[i + 1] - S->vbase[i])
            return set_error(DG_EINVAL, "source of member %d out of range", i);
        gs[i] = (int32_t)(S->vbase[i] + sources[i]);
    }
    dg_query *q = new dg_query();
    q->g = S->g;
    q->kind = Q_SSSP;
    q->source = gs[0];
    q->nsrc = S->count;
    q->gcache = &S->cache;
    if (q->srcs.ensure(S->count + 1) != DG_OK ||
        hipMemcpy(q->srcs.p, gs.data(), gs.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        q->srcs.release();
        delete q;
        return set_error(DG_ENOMEM, "source list allocation failed");
    }
    dg_query *out = nullptr;
    DG_TRY(query_attach(S->g, q, &out));
    S->q = out;
    return DG_OK;
}

static int set_stage_batch(dg_set *S, const int64_t *k, const int32_t *src, const int32_t *dst, const int32_t *w,
                           const uint8_t *op, uint32_t flags, int64_t *total, const int32_t **os,
                           const int32_t **od, const int32_t **dw, const uint8_t **dop) {
    if (!S || !k) return set_error(DG_EINVAL, "bad arguments");
    if (flags & ~(DG_DEVICE_PTRS)) return set_error(DG_EINVAL, "unknown flags");
    int64_t K = 0;
    for (int32_t i = 0; i < S->count; ++i) K += k[i] > 0 ? k[i] : 0;
    if (K > 0 && (!src || !dst || !op)) return set_error(DG_EINVAL, "null batch arrays");
    const bool dev = (flags & DG_DEVICE_PTRS) != 0;
    DG_TRY(set_translate(S, k, K, src, dst, dev, os, od));
    DG_TRY(stage_into(w, K, dev, S->stream, S->tw, dw));
    DG_TRY(stage_into(op, K, dev, S->stream, S->top, dop));
    *total = K;
    return DG_OK;
}

int dg_set_apply_sssp(dg_set *S, const int64_t *k, const int32_t *src, const int32_t *dst, const int32_t *w,
                      const uint8_t *op, uint32_t flags, dg_batch_stats *stats) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    int64_t K = 0;
    const int32_t *os, *od, *dw;
    const uint8_t *dop;
    DG_TRY(set_stage_batch(S, k, src, dst, w, op, flags, &K, &os, &od, &dw, &dop));
    if (K == 0) return DG_OK;
    int rc = apply_chunk(S->g, K, os, od, dw, dop, true, stats);
    if (rc == DG_EDEVICE) S->g->broken = true;
    return rc;
}

int dg_set_sssp_read(dg_set *S, int32_t member, int32_t *dist, int32_t *parent, uint32_t flags) {
    if (!S || !S->q || member < 0 || member >= S->count || !dist) return set_error(DG_EINVAL, "bad arguments");
    const int64_t base = S->vbase[member], nl = S->vbase[member + 1] - base;
    hipStream_t s = S->stream;
    if (flags & DG_DEVICE_PTRS) {
        hipLaunchKernelGGL(k_set_unpack, dim3(grid_for(nl)), dim3(256), 0, s, nl, S->q->key.p, base, dist, parent);
        DG_HIP(hipGetLastError());
        DG_HIP(hipStreamSynchronize(s));
        return DG_OK;
    }
    DG_TRY(S->g->ws.rbuf.ensure((size_t)nl + 1));
    int32_t *tmp = reinterpret_cast<int32_t *>(S->g->ws.rbuf.p);  // 2 nl + 2 int32
    hipLaunchKernelGGL(k_set_unpack, dim3(grid_for(nl)), dim3(256), 0, s, nl, S->q->key.p, base, tmp,
                       parent ? tmp + nl : nullptr);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(dist, tmp, nl * 4, hipMemcpyDeviceToHost, s);
    hipError_t e3 = parent ? hipMemcpyAsync(parent, tmp + nl, nl * 4, hipMemcpyDeviceToHost, s) : hipSuccess;
    hipError_t e4 = hipStreamSynchronize(s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
        return set_error(DG_EDEVICE, "set read failed");
    return DG_OK;
}

int dg_set_graph_stats(dg_set *S, int64_t *launches, int64_t *captures) {
    if (!S) return set_error(DG_EINVAL, "null set");
    if (launches) *launches = S->cache.launches;
    if (captures) *captures = S->cache.captures;
    return DG_OK;
}

int dg_autotune(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst, const int32_t *w,
                const uint8_t *op, uint32_t flags, dg_config *best, double *best_ms) {
    if (!g) return set_error(DG_EINVAL, "null graph");
    auto apply = [&]() { return dg_apply_batch(g, k, src, dst, w, op, 0, flags, nullptr); };
    return tune(g, apply, best, best_ms);
}

int dg_set_autotune(dg_set *S, const int64_t *k, const int32_t *src, const int32_t *dst, const int32_t *w,
                    const uint8_t *op, uint32_t flags, dg_config *best, double *best_ms) {
    if (!S) return set_error(DG_EINVAL, "null set");
    auto apply = [&]() { return dg_set_apply_sssp(S, k, src, dst, w, op, flags, nullptr); };
    return tune(S->g, apply, best, best_ms);
}

}  // extern "C"
