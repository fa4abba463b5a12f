// Serving loop: resident graphs, continuous batching across graphs, admission by
// device-memory budget, per-request timestamps.
//
// Each resident graph keeps a maintained PageRank and a symmetrised undirected
// copy with a maintained triangle count.  A request is one update batch for one
// graph plus one query (shortest paths from a source, PageRank, or triangles of
// the symmetrised copy).  W worker threads each own a HIP stream; a free worker
// takes the oldest waiting request of a graph no other worker holds, as soon as
// its estimated device bytes fit the budget, so requests that arrive while others
// run start as soon as a slot and memory free up and work for different graphs
// overlaps on the device.  Requests of one graph run in arrival order, so every
// result equals the result of running the same sequence alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dg_device.h"

namespace dg {

// Directed deletions (u, v) whose reverse arc (v, u) is still live: in the
// symmetrised copy the edge {u, v} stays (T4 reading: {u,v} is an edge while
// either arc is).  keep[i] = 0 for those, 1 otherwise.  perm maps the caller's
// ids to the directed graph's internal ids (null: kept as given).
__global__ void k_sym_keep(int64_t k, const int32_t *s, const int32_t *d, const uint8_t *op, const int32_t *perm,
                           const int64_t *off, const int32_t *col, const int64_t *doff, const int32_t *dcol,
                           uint8_t *keep) {
    for (int64_t i = gtid(); i < k; i += gstride()) {
        uint8_t kp = 1;
        if (op[i] == 0) {
            const int32_t u = perm ? perm[s[i]] : s[i], v = perm ? perm[d[i]] : d[i];
            int64_t p = find_sorted(col, off[v], off[v + 1], (uint32_t)u);
            bool live = p >= 0 && !((uint32_t)col[p] & DEAD);
            if (p < 0) {
                int64_t q = find_sorted(dcol, doff[v], doff[v + 1], (uint32_t)u);
                live = q >= 0 && !((uint32_t)dcol[q] & DEAD);
            }
            kp = live ? 0 : 1;
        }
        keep[i] = kp;
    }
}

int sym_keep_mask(dg_graph *g, int64_t k, const int32_t *ds, const int32_t *dd, const uint8_t *dop, uint8_t *keep) {
    if (k <= 0) return DG_OK;
    int64_t blocks = std::min<int64_t>((k + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sym_keep, dim3((unsigned)blocks), dim3(256), 0, g->stream, k, ds, dd, dop,
                       g->relabeled ? (const int32_t *)g->perm.p : nullptr, g->fwd.off.p, g->fwd.col.p,
                       g->fwd.doff.p, g->fwd.dcol.p, keep);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

}  // namespace dg

using namespace dg;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    int64_t ticket = 0;
    int32_t graph = 0, kind = 0, source = 0;
    std::vector<int32_t> src, dst, w;
    std::vector<uint8_t> op;
    void *out = nullptr;
    int64_t bytes = 0;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = DG_OK;
    bool done = false;
    uint64_t tc = 0;
    int32_t pr_iters = 0;
    int64_t applied = 0;
    char error[96] = "";  // the worker's error message when status != DG_OK
};

struct Entry {
    dg_graph *g = nullptr, *gu = nullptr;
    dg_query *pr = nullptr, *tc = nullptr;
    int32_t n = 0;
    bool busy = false;
    std::deque<Req *> fifo;
    // staging of the symmetrised-copy filter, kept across requests (a device free
    // synchronises the whole device and would serialise the workers)
    DBuf<int32_t> ss, sd;
    DBuf<uint8_t> sop, skeep;
};

}  // namespace

struct dg_server {
    dg_server_config cfg{};
    std::vector<Entry> graphs;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false, started = false;
    std::unordered_map<int64_t, Req *> reqs;
    int64_t next_ticket = 1;
    int64_t inflight_bytes = 0;
    int64_t waiting = 0;
    size_t rr = 0;  // round-robin start over graphs
    Clock::time_point t0 = Clock::now();
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// One request on one worker stream: apply, keep the symmetrised copy in step,
// answer the query.
int run_request(dg_server *S, Entry &E, Req *r, hipStream_t stream) {
    DG_TRY(dg_graph_set_stream(E.g, stream));
    DG_TRY(dg_graph_set_stream(E.gu, stream));
    const int64_t k = (int64_t)r->src.size();
    dg_batch_stats st{};
    if (k > 0) {
        DG_TRY(dg_apply_batch(E.g, k, r->src.data(), r->dst.data(), r->w.data(), r->op.data(), 0, 0, &st));
        r->applied = st.deleted + st.inserted;
        // symmetrised copy: insert {u,v}; delete {u,v} unless (v,u) is still live
        DBuf<int32_t> &ds = E.ss, &dd = E.sd;
        DBuf<uint8_t> &dop = E.sop, &keep = E.skeep;
        int rc = ds.ensure(k + 1);
        if (rc == DG_OK) rc = dd.ensure(k + 1);
        if (rc == DG_OK) rc = dop.ensure(k + 1);
        if (rc == DG_OK) rc = keep.ensure(k + 1);
        std::vector<uint8_t> hk(k);
        if (rc == DG_OK) {
            (void)hipMemcpyAsync(ds.p, r->src.data(), k * 4, hipMemcpyHostToDevice, stream);
            (void)hipMemcpyAsync(dd.p, r->dst.data(), k * 4, hipMemcpyHostToDevice, stream);
            (void)hipMemcpyAsync(dop.p, r->op.data(), k, hipMemcpyHostToDevice, stream);
            rc = sym_keep_mask(E.g, k, ds.p, dd.p, dop.p, keep.p);
        }
        if (rc == DG_OK && hipMemcpyAsync(hk.data(), keep.p, k, hipMemcpyDeviceToHost, stream) != hipSuccess)
            rc = set_error(DG_EDEVICE, "copy failed");
        if (rc == DG_OK && hipStreamSynchronize(stream) != hipSuccess) rc = set_error(DG_EDEVICE, "sync failed");
        if (rc != DG_OK) return rc;
        std::vector<int32_t> us, vs;
        std::vector<uint8_t> os;
        us.reserve(k); vs.reserve(k); os.reserve(k);
        for (int64_t i = 0; i < k; ++i) {
            if (!hk[i]) continue;
            us.push_back(r->src[i]);
            vs.push_back(r->dst[i]);
            os.push_back(r->op[i]);
        }
        if (!us.empty())
            DG_TRY(dg_apply_batch(E.gu, (int64_t)us.size(), us.data(), vs.data(), nullptr, os.data(), 0, 0, nullptr));
    }
    if (r->kind == 0) {
        DG_TRY(dg_sssp_static(E.g, r->source, static_cast<int32_t *>(r->out), nullptr, 0));
    } else if (r->kind == 1) {
        int32_t it = 0, conv = 0;
        DG_TRY(dg_pr_read(E.pr, static_cast<double *>(r->out), &it, &conv, 0));
        r->pr_iters = it;
    } else {
        DG_TRY(dg_tc_read(E.tc, &r->tc));
        if (r->out) *static_cast<uint64_t *>(r->out) = r->tc;
    }
    return DG_OK;
}

void worker(dg_server *S, size_t wi) {
    hipStream_t stream = S->streams[wi];
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        Req *r = nullptr;
        size_t gi = 0;
        while (!S->stop) {
            const size_t G = S->graphs.size();
            // oldest waiting request among idle graphs that fits the budget
            double best_t = 1e300;
            for (size_t j = 0; j < G; ++j) {
                Entry &E = S->graphs[j];
                if (E.busy || E.fifo.empty()) continue;
                Req *c = E.fifo.front();
                if (S->inflight_bytes + c->bytes > S->cfg.budget_bytes) continue;
                if (c->t_submit < best_t) {
                    best_t = c->t_submit;
                    r = c;
                    gi = j;
                }
            }
            if (r) break;
            S->cv_work.wait(lk);
        }
        if (!r) break;
        Entry &E = S->graphs[gi];
        E.fifo.pop_front();
        E.busy = true;
        S->inflight_bytes += r->bytes;
        S->waiting -= 1;
        r->t_start = S->now();
        lk.unlock();
        int rc = run_request(S, E, r, stream);
        lk.lock();
        r->t_end = S->now();
        r->status = rc;
        if (rc != DG_OK) std::snprintf(r->error, sizeof(r->error), "%s", dg_last_error());
        r->done = true;
        E.busy = false;
        S->inflight_bytes -= r->bytes;
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

int dg_server_create(const dg_server_config *cfg, dg_server **out) {
    if (!out) return set_error(DG_EINVAL, "null output");
    dg_server *S = new dg_server();
    if (cfg) S->cfg = *cfg;
    if (S->cfg.workers <= 0) S->cfg.workers = 4;
    if (S->cfg.budget_bytes <= 0) S->cfg.budget_bytes = 8ll << 30;
    if (S->cfg.max_waiting <= 0) S->cfg.max_waiting = 1 << 20;
    *out = S;
    return DG_OK;
}

int dg_server_add_graph(dg_server *S, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                        const int32_t *w, const dg_config *cfg, int32_t *graph_id) {
    if (!S || !graph_id) return set_error(DG_EINVAL, "bad arguments");
    if (S->started) return set_error(DG_ESTATE, "add graphs before dg_server_start");
    Entry E;
    E.n = n;
    DG_TRY(dg_graph_create(n, m, src, dst, w, 0, cfg, &E.g));
    // symmetrised copy: each unordered pair once
    std::vector<int64_t> keys(m);
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = std::min(src[i], dst[i]), b = std::max(src[i], dst[i]);
        keys[i] = ((int64_t)a << 32) | (uint32_t)b;
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<int32_t> us(keys.size()), vs(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
        us[i] = (int32_t)(keys[i] >> 32);
        vs[i] = (int32_t)(keys[i] & 0xffffffff);
    }
    int rc = dg_graph_create(n, (int64_t)keys.size(), us.data(), vs.data(), nullptr, DG_UNDIRECTED, cfg, &E.gu);
    if (rc == DG_OK) rc = dg_pr_attach(E.g, 0.85, 1e-9, 1000, &E.pr);
    if (rc == DG_OK) rc = dg_tc_attach(E.gu, &E.tc);
    if (rc != DG_OK) {
        if (E.g) dg_graph_destroy(E.g);
        if (E.gu) dg_graph_destroy(E.gu);
        return rc;
    }
    *graph_id = (int32_t)S->graphs.size();
    S->graphs.push_back(std::move(E));
    return DG_OK;
}

int dg_server_start(dg_server *S) {
    if (!S) return set_error(DG_EINVAL, "null server");
    if (S->started) return set_error(DG_ESTATE, "already started");
    for (int i = 0; i < S->cfg.workers; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) return set_error(DG_EDEVICE, "stream creation failed");
        S->streams.push_back(st);
    }
    S->started = true;
    S->t0 = Clock::now();
    for (int i = 0; i < S->cfg.workers; ++i) S->workers.emplace_back(worker, S, (size_t)i);
    return DG_OK;
}

int dg_server_submit(dg_server *S, const dg_request *q, int64_t *ticket) {
    if (!S || !q || !ticket) return set_error(DG_EINVAL, "bad arguments");
    if (q->graph < 0 || q->graph >= (int32_t)S->graphs.size()) return set_error(DG_EINVAL, "no such graph");
    if (q->kind < 0 || q->kind > 2) return set_error(DG_EINVAL, "unknown query kind");
    if (q->k < 0 || (q->k > 0 && (!q->src || !q->dst || !q->op))) return set_error(DG_EINVAL, "bad batch");
    const int32_t n = S->graphs[q->graph].n;
    if (q->kind == 0 && (q->source < 0 || q->source >= n)) return set_error(DG_EINVAL, "bad source");
    if (q->kind != 2 && !q->out) return set_error(DG_EINVAL, "null output buffer");
    Req *r = new Req();
    r->graph = q->graph;
    r->kind = q->kind;
    r->source = q->source;
    r->out = q->out;
    r->src.assign(q->src, q->src + q->k);
    r->dst.assign(q->dst, q->dst + q->k);
    r->op.assign(q->op, q->op + q->k);
    if (q->w) r->w.assign(q->w, q->w + q->k);
    else r->w.assign(q->k, 1);
    // device bytes while the request runs: batch staging and sort buffers
    // (about 96 B per update, twice for the symmetrised copy) plus the answer
    // (SSSP keys + unpack 16 B per vertex, PageRank 16 B per vertex)
    r->bytes = 192 * q->k + (q->kind == 2 ? 0 : 16ll * n) + (1 << 20);
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->bytes > S->cfg.budget_bytes) {
        delete r;
        return set_error(DG_EBUDGET, "request needs more device memory than the whole budget");
    }
    if (S->waiting >= S->cfg.max_waiting) {
        delete r;
        return set_error(DG_EBUSY, "too many waiting requests");
    }
    r->ticket = S->next_ticket++;
    r->t_submit = S->now();
    S->reqs[r->ticket] = r;
    S->graphs[q->graph].fifo.push_back(r);
    S->waiting += 1;
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return DG_OK;
}

static void fill_result(const Req *r, dg_result *res) {
    std::memset(res, 0, sizeof(*res));
    res->status = r->status;
    res->t_submit = r->t_submit;
    res->t_start = r->t_start;
    res->t_end = r->t_end;
    res->applied = r->applied;
    res->tc = r->tc;
    res->pr_iters = r->pr_iters;
    std::memcpy(res->error, r->error, sizeof(res->error));
}

int dg_server_wait(dg_server *S, int64_t ticket, double timeout_s, dg_result *res) {
    if (!S || !res) return set_error(DG_EINVAL, "bad arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(DG_ENOTFOUND, "unknown ticket");
    Req *r = it->second;
    auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                                       timeout_s < 0 ? 1e9 : timeout_s));
    while (!r->done)
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done)
            return set_error(DG_ENOTFOUND, "not finished before the timeout");
    fill_result(r, res);
    S->reqs.erase(it);
    delete r;
    return DG_OK;
}

int dg_server_poll(dg_server *S, int64_t ticket, dg_result *res) { return dg_server_wait(S, ticket, 0.0, res); }

int dg_server_stats(dg_server *S, int64_t *waiting, int64_t *inflight_bytes) {
    if (!S) return set_error(DG_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (waiting) *waiting = S->waiting;
    if (inflight_bytes) *inflight_bytes = S->inflight_bytes;
    return DG_OK;
}

int dg_server_destroy(dg_server *S) {
    if (!S) return set_error(DG_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->reqs) delete kv.second;
    for (auto &E : S->graphs) {
        for (auto *r : E.fifo) (void)r;  // owned by reqs (already deleted)
        if (E.g) dg_graph_destroy(E.g);
        if (E.gu) dg_graph_destroy(E.gu);
        E.ss.release(); E.sd.release(); E.sop.release(); E.skeep.release();
    }
    for (auto st : S->streams) (void)hipStreamDestroy(st);
    delete S;
    return DG_OK;
}

}  // extern "C"
