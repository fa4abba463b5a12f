// C ABI entry points (declared in include/dg.h): argument checks, handle life
// cycle, chunking of update batches, and snapshots.  All computation happens in
// the kernels of graph.hip, sssp.hip, pagerank.hip and tc.hip.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "dg_internal.h"

namespace dg {

static thread_local char g_err[1024] = "";
static void *(*g_alloc)(size_t, void *) = nullptr;
static void (*g_free)(void *, void *) = nullptr;
static void *g_ctx = nullptr;
static std::atomic<int> g_live_graphs{0};

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void *dmalloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (g_alloc) return g_alloc(bytes, g_ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dfree(void *p) {
    if (!p) return;
    if (g_free) g_free(p, g_ctx);
    else (void)hipFree(p);
}

static dg_config defaults(const dg_config *c) {
    dg_config r{};
    if (c) r = *c;
    if (r.merge_threshold == 0.0) r.merge_threshold = 0.05;
    if (r.pr_tol_scale <= 0.0) r.pr_tol_scale = 1.0;
    return r;
}

// Copy a host int32 array to a fresh device buffer (or pass device pointers through).
template <class T>
static int stage(const T *p, int64_t n, bool dev, hipStream_t s, DBuf<T> &buf, const T **out) {
    if (!p || dev) {
        *out = p;
        return DG_OK;
    }
    DG_TRY(buf.ensure((size_t)n + 1));
    if (n > 0) DG_HIP(hipMemcpyAsync(buf.p, p, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
    *out = buf.p;
    return DG_OK;
}

static int check_graph(dg_graph *g) {
    if (!g) return set_error(DG_EINVAL, "null graph");
    if (g->broken) return set_error(DG_ESTATE, "graph handle unusable after an earlier device error");
    return DG_OK;
}

static int mark_device_error(dg_graph *g, int rc) {
    if (rc == DG_EDEVICE && g) g->broken = true;
    return rc;
}

// ---- snapshots --------------------------------------------------------------------------

template <class T>
static int snap_save(dg_snapshot *sn, const DBuf<T> &b, size_t count, hipStream_t s) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void *p = dmalloc(bytes);
    if (!p) return set_error(DG_ENOMEM, "snapshot allocation failed");
    sn->bufs.push_back({p, count * sizeof(T)});
    if (count) DG_HIP(hipMemcpyAsync(p, b.p, count * sizeof(T), hipMemcpyDeviceToDevice, s));
    return DG_OK;
}

template <class T>
static int snap_load(const dg_snapshot *sn, size_t &idx, DBuf<T> &b, hipStream_t s) {
    const auto &e = sn->bufs[idx++];
    size_t count = e.second / sizeof(T);
    DG_TRY(b.ensure(count + 1));
    if (count) DG_HIP(hipMemcpyAsync(b.p, e.first, e.second, hipMemcpyDeviceToDevice, s));
    return DG_OK;
}

static int64_t ntiles(int64_t m) { return (m + TILE - 1) / TILE + 2; }

static int snap_dir(dg_snapshot *sn, const Dir &d, int32_t n, hipStream_t s) {
    DG_TRY(snap_save(sn, d.off, n + 1, s));
    DG_TRY(snap_save(sn, d.col, d.m, s));
    DG_TRY(snap_save(sn, d.w, d.m, s));
    DG_TRY(snap_save(sn, d.doff, n + 1, s));
    DG_TRY(snap_save(sn, d.dkey, d.dm, s));
    DG_TRY(snap_save(sn, d.dcol, d.dm, s));
    DG_TRY(snap_save(sn, d.dw, d.dm, s));
    DG_TRY(snap_save(sn, d.deg, n, s));
    DG_TRY(snap_save(sn, d.ntomb, n, s));
    DG_TRY(snap_save(sn, d.ttomb, ntiles(d.m), s));
    sn->scalars.push_back(d.m);
    sn->scalars.push_back(d.dm);
    sn->scalars.push_back(d.tomb_base);
    sn->scalars.push_back(d.tomb_diff);
    return DG_OK;
}

static int load_dir(const dg_snapshot *sn, size_t &idx, size_t &si, Dir &d, hipStream_t s) {
    DG_TRY(snap_load(sn, idx, d.off, s));
    DG_TRY(snap_load(sn, idx, d.col, s));
    DG_TRY(snap_load(sn, idx, d.w, s));
    DG_TRY(snap_load(sn, idx, d.doff, s));
    DG_TRY(snap_load(sn, idx, d.dkey, s));
    DG_TRY(snap_load(sn, idx, d.dcol, s));
    DG_TRY(snap_load(sn, idx, d.dw, s));
    DG_TRY(snap_load(sn, idx, d.deg, s));
    DG_TRY(snap_load(sn, idx, d.ntomb, s));
    DG_TRY(snap_load(sn, idx, d.ttomb, s));
    d.m = sn->scalars[si++];
    d.dm = sn->scalars[si++];
    d.tomb_base = sn->scalars[si++];
    d.tomb_diff = sn->scalars[si++];
    return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" {

const char *dg_last_error(void) { return dg::g_err; }

int dg_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
    if (g_live_graphs.load() > 0) return set_error(DG_ESTATE, "allocator must be set before any graph exists");
    if ((alloc == nullptr) != (free_fn == nullptr)) return set_error(DG_EINVAL, "alloc and free come together");
    g_alloc = alloc;
    g_free = free_fn;
    g_ctx = ctx;
    return DG_OK;
}

int dg_graph_create(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *w,
                    uint32_t flags, const dg_config *cfg, dg_graph **out) {
    if (!out) return set_error(DG_EINVAL, "null output handle");
    *out = nullptr;
    if (n <= 0 || n > (1 << 30)) return set_error(DG_EINVAL, "n must be in [1, 2^30]");
    if (m < 0 || (m > 0 && (!src || !dst))) return set_error(DG_EINVAL, "bad edge list");
    if (flags & ~(DG_UNDIRECTED | DG_DEVICE_PTRS)) return set_error(DG_EINVAL, "unknown flags");
    dg_graph *g = new dg_graph();
    g->n = n;
    g->undirected = (flags & DG_UNDIRECTED) != 0;
    g->cfg = defaults(cfg);
    g->relabeled = g->cfg.vertex_order == 0;
    g->rev = g->undirected ? &g->fwd : &g->rev_own;
    int rc = ws_init(g);
    const bool dev = (flags & DG_DEVICE_PTRS) != 0;
    DBuf<int32_t> bs, bd, bw;
    const int32_t *ds = nullptr, *dd = nullptr, *dw = nullptr;
    if (rc == DG_OK) rc = stage(src, m, dev, g->stream, bs, &ds);
    if (rc == DG_OK) rc = stage(dst, m, dev, g->stream, bd, &dd);
    if (rc == DG_OK) rc = stage(w, m, dev, g->stream, bw, &dw);
    if (rc == DG_OK) rc = graph_build(g, m, ds, dd, dw);
    bs.release();
    bd.release();
    bw.release();
    if (rc != DG_OK) {
        char keep[1024];
        std::strncpy(keep, g_err, sizeof(keep) - 1);
        keep[sizeof(keep) - 1] = 0;
        dir_free(g->fwd);
        dir_free(g->rev_own);
        ws_free(g);
        delete g;
        std::strncpy(g_err, keep, sizeof(g_err));
        return rc;
    }
    ++g_live_graphs;
    *out = g;
    return DG_OK;
}

// Device and pinned memory of a query, then the query itself.
static void query_free(dg_query *q) {
    q->key.release(); q->inval.release(); q->x.release(); q->xn.release(); q->contrib.release(); q->res.release();
    q->qcnt.release(); q->srcs.release(); q->gstamp.release(); q->gfar.release();
    if (q->hpin) (void)hipHostFree(q->hpin);
    if (q->own_cache) {
        graph_cache_clear(q->own_cache);
        delete q->own_cache;
    }
    delete q;
}

int dg_graph_destroy(dg_graph *g) {
    if (!g) return set_error(DG_EINVAL, "null graph");
    for (dg_query *q : g->queries) {
        query_free(q);
    }
    g->queries.clear();
    (void)hipStreamSynchronize(g->stream);
    dir_free(g->fwd);
    dir_free(g->rev_own);
    ws_free(g);
    delete g;
    --g_live_graphs;
    return DG_OK;
}

int dg_graph_set_stream(dg_graph *g, void *stream) {
    DG_TRY(check_graph(g));
    DG_HIP(hipStreamSynchronize(g->stream));
    g->stream = static_cast<hipStream_t>(stream);
    return DG_OK;
}

int dg_graph_info(dg_graph *g, int32_t *n, int64_t *m_live, int64_t *diff, int64_t *tomb) {
    if (!g) return set_error(DG_EINVAL, "null graph");
    if (n) *n = g->n;
    if (m_live) *m_live = g->undirected ? g->m_live / 2 : g->m_live;
    if (diff) *diff = g->fwd.dm;
    if (tomb) *tomb = g->fwd.tomb_base;
    return DG_OK;
}

int dg_graph_export(dg_graph *g, int64_t *m, int32_t *src, int32_t *dst, int32_t *w) {
    DG_TRY(check_graph(g));
    if (!m || (src && !dst)) return set_error(DG_EINVAL, "bad export arguments");
    return mark_device_error(g, graph_export(g, m, src, dst, w));
}

int dg_graph_merge(dg_graph *g) {
    DG_TRY(check_graph(g));
    return mark_device_error(g, graph_merge(g));
}

int dg_apply_batch(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst, const int32_t *w,
                   const uint8_t *op, int64_t batch_size, uint32_t flags, dg_batch_stats *stats) {
    DG_TRY(check_graph(g));
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (flags & ~(DG_DEVICE_PTRS | DG_INCREMENTAL | DG_DECREMENTAL)) return set_error(DG_EINVAL, "unknown flags");
    const uint32_t mode = flags & (DG_INCREMENTAL | DG_DECREMENTAL);
    if (mode == (DG_INCREMENTAL | DG_DECREMENTAL))
        return set_error(DG_EINVAL, "DG_INCREMENTAL and DG_DECREMENTAL together");
    const int expect = mode == DG_INCREMENTAL ? 1 : (mode == DG_DECREMENTAL ? 0 : -1);
    if (k < 0 || (k > 0 && (!src || !dst || (!op && expect < 0)))) return set_error(DG_EINVAL, "bad batch arguments");
    if (k > INT32_MAX / 4) return set_error(DG_EINVAL, "batch chunk too large");
    const bool dev = (flags & DG_DEVICE_PTRS) != 0;
    // a mode without an op array: every update gets the mode's op
    std::vector<uint8_t> hop;
    DBuf<uint8_t> dop;
    if (!op && k > 0) {
        if (dev) {
            DG_TRY(dop.ensure((size_t)k));
            DG_HIP(hipMemsetAsync(dop.p, expect, (size_t)k, g->stream));
            op = dop.p;
        } else {
            hop.assign((size_t)k, (uint8_t)expect);
            op = hop.data();
        }
    }
    const int64_t bs = batch_size <= 0 ? std::max<int64_t>(k, 1) : batch_size;
    for (int64_t o = 0; o < k; o += bs) {
        int64_t kk = std::min(bs, k - o);
        int rc = apply_chunk(g, kk, src + o, dst + o, w ? w + o : nullptr, op + o, dev, stats, expect);
        if (rc != DG_OK) return mark_device_error(g, rc);
    }
    return DG_OK;
}

int dg_snapshot_save(dg_graph *g, dg_snapshot **out) {
    DG_TRY(check_graph(g));
    if (!out) return set_error(DG_EINVAL, "null output");
    dg_snapshot *sn = new dg_snapshot();
    sn->g = g;
    hipStream_t s = g->stream;
    int rc = snap_dir(sn, g->fwd, g->n, s);
    if (rc == DG_OK && !g->undirected) rc = snap_dir(sn, g->rev_own, g->n, s);
    sn->scalars.push_back(g->m_live);
    for (dg_query *q : g->queries) {
        if (rc != DG_OK) break;
        sn->queries.push_back(q);
        if (q->kind == Q_SSSP) rc = snap_save(sn, q->key, g->n, s);
        else if (q->kind == Q_PR) {
            rc = snap_save(sn, q->x, g->n, s);
            if (rc == DG_OK) rc = snap_save(sn, q->contrib, g->n, s);
            if (rc == DG_OK) rc = snap_save(sn, q->res, q->res.p ? g->n : 0, s);
            sn->scalars.push_back(q->last_iters);
            sn->scalars.push_back(q->converged);
        } else sn->scalars.push_back((int64_t)q->tc);
    }
    if (rc == DG_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_error(DG_EDEVICE, "snapshot copy failed");
    if (rc != DG_OK) {
        dg_snapshot_free(sn);
        return rc;
    }
    *out = sn;
    return DG_OK;
}

int dg_snapshot_restore(dg_graph *g, const dg_snapshot *sn) {
    DG_TRY(check_graph(g));
    if (!sn || sn->g != g) return set_error(DG_EINVAL, "snapshot belongs to another graph");
    if (sn->queries != g->queries) return set_error(DG_ESTATE, "queries changed since the snapshot");
    hipStream_t s = g->stream;
    size_t idx = 0, si = 0;
    DG_TRY(load_dir(sn, idx, si, g->fwd, s));
    if (!g->undirected) DG_TRY(load_dir(sn, idx, si, g->rev_own, s));
    g->m_live = sn->scalars[si++];
    for (dg_query *q : g->queries) {
        if (q->kind == Q_SSSP) DG_TRY(snap_load(sn, idx, q->key, s));
        else if (q->kind == Q_PR) {
            DG_TRY(snap_load(sn, idx, q->x, s));
            DG_TRY(snap_load(sn, idx, q->contrib, s));
            if (sn->bufs[idx].second > 0) DG_TRY(snap_load(sn, idx, q->res, s));
            else ++idx;
            q->last_iters = (int32_t)sn->scalars[si++];
            q->converged = (int32_t)sn->scalars[si++];
        } else q->tc = (uint64_t)sn->scalars[si++];
    }
    DG_HIP(hipStreamSynchronize(s));
    return DG_OK;
}

int dg_snapshot_free(dg_snapshot *sn) {
    if (!sn) return DG_OK;
    for (auto &b : sn->bufs) dfree(b.first);
    delete sn;
    return DG_OK;
}

// ---- queries ---------------------------------------------------------------------------------

static int attach(dg_graph *g, dg_query *q, dg_query **out) {
    int rc = q->kind == Q_SSSP ? sssp_init(q) : (q->kind == Q_PR ? pr_init(q) : tc_count_static(g, &q->tc));
    if (rc != DG_OK) {
        query_free(q);
        return mark_device_error(g, rc);
    }
    g->queries.push_back(q);
    *out = q;
    return DG_OK;
}

int dg_sssp_attach(dg_graph *g, int32_t source, dg_query **q) {
    DG_TRY(check_graph(g));
    if (!q || source < 0 || source >= g->n) return set_error(DG_EINVAL, "bad source");
    int32_t iv = source;
    DG_TRY(vertex_in(g, source, &iv));
    dg_query *x = new dg_query();
    x->g = g;
    x->kind = Q_SSSP;
    x->source = iv;
    return attach(g, x, q);
}

int dg_pr_attach(dg_graph *g, double damping, double tol, int32_t max_iter, dg_query **q) {
    DG_TRY(check_graph(g));
    if (!q || !(damping > 0.0 && damping < 1.0) || !(tol > 0.0) || max_iter < 1)
        return set_error(DG_EINVAL, "bad PageRank parameters");
    dg_query *x = new dg_query();
    x->g = g;
    x->kind = Q_PR;
    x->damping = damping;
    x->tol = tol;
    x->max_iter = max_iter;
    return attach(g, x, q);
}

int dg_tc_attach(dg_graph *g, dg_query **q) {
    DG_TRY(check_graph(g));
    if (!q) return set_error(DG_EINVAL, "null output");
    if (!g->undirected) return set_error(DG_EINVAL, "triangle counting needs an undirected graph");
    dg_query *x = new dg_query();
    x->g = g;
    x->kind = Q_TC;
    return attach(g, x, q);
}

int dg_query_detach(dg_query *q) {
    if (!q) return set_error(DG_EINVAL, "null query");
    dg_graph *g = q->g;
    auto it = std::find(g->queries.begin(), g->queries.end(), q);
    if (it == g->queries.end()) return set_error(DG_EINVAL, "query not attached");
    g->queries.erase(it);
    (void)hipStreamSynchronize(g->stream);
    query_free(q);
    return DG_OK;
}

// ---- checkpoint / resume of query state ---------------------------------------------------

namespace {
// Host byte layout of an exported query: this header, then the payload (SSSP:
// int32 dist[n] and int32 parent[n]; PageRank: double x[n]; triangles: none),
// everything in the caller's vertex ids.
struct QueryBlob {
    uint32_t magic;
    int32_t kind;
    int32_t n;
    int32_t source;     // SSSP: caller's id
    int64_t m_live;     // live edges of the graph at export
    double damping, tol;
    int32_t max_iter, last_iters, converged, reserved;
    uint64_t tc;
};
constexpr uint32_t BLOB_MAGIC = 0x31515344u;  // "DSQ1"

int64_t blob_payload(int kind, int32_t n) {
    return kind == Q_SSSP ? 8 * (int64_t)n : (kind == Q_PR ? 8 * (int64_t)n : 0);
}
}  // namespace

int dg_query_export(dg_query *q, void *buf, int64_t *bytes) {
    if (!q || !bytes) return set_error(DG_EINVAL, "null query or size");
    dg_graph *g = q->g;
    DG_TRY(check_graph(g));
    if (q->nsrc > 0) return set_error(DG_EINVAL, "queries of a graph set are not exported");
    const int64_t need = (int64_t)sizeof(QueryBlob) + blob_payload(q->kind, g->n);
    if (!buf) {
        *bytes = need;
        return DG_OK;
    }
    if (*bytes < need) return set_error(DG_EINVAL, "export buffer holds %lld bytes, %lld needed",
                                        (long long)*bytes, (long long)need);
    QueryBlob h{};
    h.magic = BLOB_MAGIC;
    h.kind = q->kind;
    h.n = g->n;
    h.m_live = g->undirected ? g->m_live / 2 : g->m_live;
    h.damping = q->damping;
    h.tol = q->tol;
    h.max_iter = q->max_iter;
    h.last_iters = q->last_iters;
    h.converged = q->converged;
    h.tc = q->tc;
    h.source = q->source;
    if (q->kind == Q_SSSP && g->relabeled) {
        int32_t c = 0;
        DG_HIP(hipMemcpy(&c, g->iperm.p + q->source, 4, hipMemcpyDeviceToHost));
        h.source = c;
    }
    char *out = static_cast<char *>(buf);
    std::memcpy(out, &h, sizeof(h));
    int rc = DG_OK;
    if (q->kind == Q_SSSP) {
        int32_t *dist = reinterpret_cast<int32_t *>(out + sizeof(h));
        rc = sssp_read(q, dist, dist + g->n, false);
    } else if (q->kind == Q_PR) {
        rc = pr_export(q, reinterpret_cast<double *>(out + sizeof(h)));
    }
    if (rc == DG_OK) *bytes = need;
    return mark_device_error(g, rc);
}

int dg_query_import(dg_graph *g, const void *buf, int64_t bytes, dg_query **q) {
    DG_TRY(check_graph(g));
    if (!buf || !q || bytes < (int64_t)sizeof(QueryBlob)) return set_error(DG_EINVAL, "bad import arguments");
    QueryBlob h;
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != BLOB_MAGIC || (h.kind != Q_SSSP && h.kind != Q_PR && h.kind != Q_TC))
        return set_error(DG_EINVAL, "not an exported query");
    if (bytes < (int64_t)sizeof(QueryBlob) + blob_payload(h.kind, h.n))
        return set_error(DG_EINVAL, "import buffer shorter than its query");
    const int64_t m_live = g->undirected ? g->m_live / 2 : g->m_live;
    if (h.n != g->n || h.m_live != m_live)
        return set_error(DG_EINVAL, "query exported from another graph (n %d, %lld edges; this graph: n %d, %lld "
                                    "edges)", h.n, (long long)h.m_live, g->n, (long long)m_live);
    const char *payload = static_cast<const char *>(buf) + sizeof(h);
    dg_query *x = new dg_query();
    x->g = g;
    x->kind = static_cast<QueryKind>(h.kind);
    int rc = DG_OK;
    if (h.kind == Q_SSSP) {
        if (h.source < 0 || h.source >= g->n) rc = set_error(DG_EINVAL, "bad source in the import");
        int32_t iv = h.source;
        if (rc == DG_OK) rc = vertex_in(g, h.source, &iv);
        x->source = iv;
        const int32_t *dist = reinterpret_cast<const int32_t *>(payload);
        if (rc == DG_OK) rc = sssp_import(x, dist, dist + g->n);
    } else if (h.kind == Q_PR) {
        if (!(h.damping > 0.0 && h.damping < 1.0) || !(h.tol > 0.0) || h.max_iter < 1)
            rc = set_error(DG_EINVAL, "bad PageRank parameters in the import");
        x->damping = h.damping;
        x->tol = h.tol;
        x->max_iter = h.max_iter;
        if (rc == DG_OK) rc = pr_import(x, reinterpret_cast<const double *>(payload));
    } else {
        if (!g->undirected) rc = set_error(DG_EINVAL, "triangle counting needs an undirected graph");
        x->tc = h.tc;
    }
    if (rc != DG_OK) {
        query_free(x);
        return mark_device_error(g, rc);
    }
    g->queries.push_back(x);
    *q = x;
    return DG_OK;
}

int dg_sssp_read(dg_query *q, int32_t *dist, int32_t *parent, uint32_t flags) {
    if (!q || q->kind != Q_SSSP) return set_error(DG_EINVAL, "not a shortest-path query");
    DG_TRY(check_graph(q->g));
    if (!dist) return set_error(DG_EINVAL, "null dist");
    return mark_device_error(q->g, sssp_read(q, dist, parent, (flags & DG_DEVICE_PTRS) != 0));
}

int dg_pr_read(dg_query *q, double *rank, int32_t *iters, int32_t *converged, uint32_t flags) {
    if (!q || q->kind != Q_PR) return set_error(DG_EINVAL, "not a PageRank query");
    DG_TRY(check_graph(q->g));
    if (!rank) return set_error(DG_EINVAL, "null rank");
    if (iters) *iters = q->last_iters;
    if (converged) *converged = q->converged;
    return mark_device_error(q->g, pr_read(q, rank, (flags & DG_DEVICE_PTRS) != 0));
}

int dg_pr_read_noalloc(dg_query *q, double *rank, int32_t *iters, int32_t *converged, uint32_t flags) {
    if (!q || q->kind != Q_PR) return set_error(DG_EINVAL, "not a PageRank query");
    DG_TRY(check_graph(q->g));
    if (!rank) return set_error(DG_EINVAL, "null rank");
    if (flags & ~DG_DEVICE_PTRS) return set_error(DG_EINVAL, "unknown flags");
    if (iters) *iters = q->last_iters;
    if (converged) *converged = q->converged;
    return mark_device_error(q->g, pr_read_noalloc(q, rank, (flags & DG_DEVICE_PTRS) != 0));
}

int dg_pr_gather_floor(dg_graph *g, int32_t reps, double *us) {
    DG_TRY(check_graph(g));
    if (!us || reps < 1) return set_error(DG_EINVAL, "gather floor needs reps >= 1 and an output");
    return mark_device_error(g, pr_gather_floor(g, reps, us));
}

int dg_tc_read(dg_query *q, uint64_t *count) {
    if (!q || q->kind != Q_TC || !count) return set_error(DG_EINVAL, "not a triangle-count query");
    *count = q->tc;
    return DG_OK;
}

// ---- sort and scan primitives ---------------------------------------------------------------

namespace {
std::mutex g_prim_mu;
SortWork g_prim_ws;
int64_t *g_prim_err = nullptr;

int prim_begin(hipStream_t s) {
    if (!g_prim_err) {
        g_prim_err = static_cast<int64_t *>(dmalloc(sizeof(int64_t)));
        if (!g_prim_err) return set_error(DG_ENOMEM, "error word allocation failed");
        DG_TRY(fill_i64(g_prim_err, 0, 1, s));
    }
    return DG_OK;
}

int prim_end(hipStream_t s) {
    int64_t e = 0;
    DG_HIP(hipMemcpyAsync(&e, g_prim_err, sizeof(e), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    if (e) return set_error(DG_EDEVICE, "sort or scan look-back did not finish (internal error)");
    return DG_OK;
}
}  // namespace

int dg_sort_pairs(const uint64_t *kin, uint64_t *kout, const int32_t *vin, int32_t *vout, int64_t n, int32_t bits,
                  void *stream) {
    if (n < 0 || (n > 0 && (!kin || !kout || !vin || !vout))) return set_error(DG_EINVAL, "bad sort arguments");
    if (bits < 1 || bits > 64) return set_error(DG_EINVAL, "bits must be in [1, 64]");
    if (n > 0 && ((const void *)kin == (const void *)kout || (const void *)vin == (const void *)vout))
        return set_error(DG_EINVAL, "sort outputs must not alias its inputs");
    std::lock_guard<std::mutex> lock(g_prim_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DG_TRY(prim_begin(s));
    DG_TRY(radix_sort_pairs(s, g_prim_ws, kin, kout, vin, vout, n, bits, g_prim_err));
    return prim_end(s);
}

int dg_scan_exclusive(const int64_t *in, int64_t *out, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return set_error(DG_EINVAL, "bad scan arguments");
    std::lock_guard<std::mutex> lock(g_prim_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DG_TRY(prim_begin(s));
    DG_TRY(scan_excl_i64(s, g_prim_ws, in, out, n, g_prim_err));
    return prim_end(s);
}

int dg_sssp_static(dg_graph *g, int32_t source, int32_t *dist, int32_t *parent, uint32_t flags) {
    DG_TRY(check_graph(g));
    if (source < 0 || source >= g->n || !dist) return set_error(DG_EINVAL, "bad arguments");
    DBuf<uint64_t> &key = g->ws.skey;
    DG_TRY(key.ensure((size_t)g->n + 1));
    int32_t iv = source;
    DG_TRY(vertex_in(g, source, &iv));
    int rc = sssp_static_solve(g, key.p, iv, nullptr);
    if (rc == DG_OK) {
        dg_query tmp;
        tmp.g = g;
        tmp.key.p = key.p;
        tmp.key.cap = key.cap;
        rc = sssp_read(&tmp, dist, parent, (flags & DG_DEVICE_PTRS) != 0);
        tmp.key.p = nullptr;
        tmp.key.cap = 0;
    }
    return mark_device_error(g, rc);
}

int dg_pr_static(dg_graph *g, double damping, double tol, int32_t max_iter, double *rank, int32_t *iters,
                 uint32_t flags) {
    DG_TRY(check_graph(g));
    if (!rank || !(damping > 0.0 && damping < 1.0) || !(tol > 0.0) || max_iter < 1)
        return set_error(DG_EINVAL, "bad PageRank parameters");
    DBuf<double> &x = g->ws.sx, &c = g->ws.sc, &xn = g->ws.sxn;
    int rc = x.ensure((size_t)g->n + 1);
    if (rc == DG_OK) rc = c.ensure((size_t)g->n + 1);
    if (rc == DG_OK) rc = xn.ensure((size_t)g->n + 1);
    int32_t it = 0, conv = 0;
    if (rc == DG_OK) rc = pr_static_solve(g, damping, tol * g->cfg.pr_tol_scale, max_iter, x.p, c.p, xn.p, &it, &conv);
    if (rc == DG_OK) rc = pr_normalize(g, x.p, rank, (flags & DG_DEVICE_PTRS) != 0);
    if (iters) *iters = it;
    return mark_device_error(g, rc);
}

int dg_tc_static(dg_graph *g, uint64_t *count) {
    DG_TRY(check_graph(g));
    if (!count) return set_error(DG_EINVAL, "null count");
    if (!g->undirected) return set_error(DG_EINVAL, "triangle counting needs an undirected graph");
    return mark_device_error(g, tc_count_static(g, count));
}

}  // extern "C"

namespace dg {

// Build a directed graph from device edge arrays on a given stream (batched sets).
int graph_create_dev(int32_t n, int64_t m, const int32_t *ds, const int32_t *dd, const int32_t *dw,
                     const dg_config *cfg, hipStream_t stream, dg_graph **out) {
    *out = nullptr;
    if (n <= 0 || n > (1 << 30)) return set_error(DG_EINVAL, "n must be in [1, 2^30]");
    dg_graph *g = new dg_graph();
    g->n = n;
    g->cfg = defaults(cfg);
    g->rev = &g->rev_own;
    g->stream = stream;
    int rc = ws_init(g);
    if (rc == DG_OK) rc = graph_build(g, m, ds, dd, dw);
    if (rc != DG_OK) {
        dir_free(g->fwd);
        dir_free(g->rev_own);
        ws_free(g);
        delete g;
        return rc;
    }
    ++g_live_graphs;
    *out = g;
    return DG_OK;
}

int query_attach(dg_graph *g, dg_query *q, dg_query **out) { return attach(g, q, out); }

}  // namespace dg
