// Persistent, launch-once SSSP fixed points on a device work queue.
//
// The frontier-step drivers of sssp.hip synchronise with the host after every
// step (the paper's fixedPoint loop copies a `finished` flag back each time,
// Section 5.3).  On high-diameter graphs and on large sets of small graphs the
// number of steps makes that round trip dominate, so this file runs the same
// relaxations (the Min of the Incremental listing, the tree cut of the
// Decremental listing) as asynchronous worklist algorithms inside a single
// kernel launch:
//
//   * a ring queue of items (vertex << 32 | chunk; chunk = ~0 means "the whole
//     row") with head / tail / done counters;
//   * a wave claims up to 64 items, expands their rows with the in-wave
//     load-balanced walk, enqueues improved vertices (one per vertex while it is
//     queued: in-queue flags), then adds the claimed count to `done`;
//   * rows longer than heavy_deg are re-enqueued as chunk items so hubs spread
//     over many waves;
//   * a wave leaves when it reads done == tail (done first, then tail: every
//     item counted in tail either is finished or keeps done below tail), so no
//     item is lost and termination does not depend on all workgroups being
//     resident at once.
// Every wait (empty queue, slot not yet written) checks an error flag and a spin
// limit, so a wave always leaves the loop.
#include <algorithm>
#include <functional>
#include <vector>

#include "traverse.h"

namespace dg {

enum { WQ_HEAD = 0, WQ_TAIL = 1, WQ_DONE = 2, WQ_ERR = 3, WQ_LIST = 4, WQ_NCTR = 8 };
// Second block of counters (not cleared between the phases of one update):
// the cut-list length carried into the push phase, then the tallies of arcs
// examined and items processed by the cut and push kernels.
enum { WT_LIST = WQ_NCTR, WT_EDGES = WQ_NCTR + 1, WT_ITEMS = WQ_NCTR + 2, WT_N = 3 };
constexpr uint32_t WHOLE = 0xFFFFFFFFu;
constexpr int64_t SPIN_LIMIT = 1ll << 22;  // a few seconds of polling (a legitimate wait is microseconds)

struct WorkQ {
    int64_t *q;
    uint64_t *seq;
    int64_t cap;
    int64_t margin;           // claimed-but-unread items at most (64 per wave of the grid)
    unsigned long long *ctr;  // WQ_* counters
    unsigned long long budget;  // items one run may claim in total (bounds pathological schedules)
};

__device__ __forceinline__ unsigned long long ld_acq(unsigned long long *p) {
    return __atomic_load_n(p, __ATOMIC_ACQUIRE);
}

// Wave-aggregated enqueue of `item` from the lanes where p is true.
__device__ __forceinline__ void wq_push(const WorkQ &wq, bool p, int64_t item) {
    uint64_t b = ballot(p);
    if (!b) return;
    int leader = __ffsll((long long)b) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(&wq.ctr[WQ_TAIL], (unsigned long long)__popcll(b));
    base = __shfl(base, leader, WAVE);
    if (p) {
        unsigned long long idx = base + __popcll(b & lanemask_lt());
        // capacity: the slot must not hold an item that has not been read yet
        if ((long long)(idx - ld_acq(&wq.ctr[WQ_HEAD])) >= wq.cap - wq.margin) {
            atomicOr(&wq.ctr[WQ_ERR], 1ull);
        } else {
            int64_t slot = (int64_t)(idx % (unsigned long long)wq.cap);
            wq.q[slot] = item;
            __threadfence();
            __atomic_store_n(&wq.seq[slot], (uint64_t)(idx + 1), __ATOMIC_RELEASE);
        }
    }
}

// Claim up to 64 items; returns false when the queue is drained (or on error).
__device__ __forceinline__ bool wq_claim(const WorkQ &wq, unsigned long long &h, int &cnt) {
    int ex = 0;
    unsigned long long hh = 0;
    int c = 0;
    if (lane_id() == 0) {
        for (int64_t spin = 0;; ++spin) {
            if (ld_acq(&wq.ctr[WQ_ERR])) { ex = 1; break; }
            unsigned long long a = ld_acq(&wq.ctr[WQ_HEAD]);
            unsigned long long t = ld_acq(&wq.ctr[WQ_TAIL]);
            if (a >= wq.budget) { atomicOr(&wq.ctr[WQ_ERR], 8ull); ex = 1; break; }
            if (a < t) {
                unsigned long long take = t - a < 64 ? t - a : 64;
                if (atomicCAS(&wq.ctr[WQ_HEAD], a, a + take) == a) {
                    hh = a;
                    c = (int)take;
                    break;
                }
                continue;
            }
            unsigned long long d = ld_acq(&wq.ctr[WQ_DONE]);
            t = ld_acq(&wq.ctr[WQ_TAIL]);
            if (d == t) { ex = 1; break; }
            if (spin > SPIN_LIMIT) { atomicOr(&wq.ctr[WQ_ERR], 2ull); ex = 1; break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    ex = __shfl(ex, 0, WAVE);
    if (ex) return false;
    h = __shfl(hh, 0, WAVE);
    cnt = __shfl(c, 0, WAVE);
    return true;
}

// Read a claimed item (waits for its producer's write).
__device__ __forceinline__ int64_t wq_read(const WorkQ &wq, unsigned long long idx, bool &ok) {
    int64_t slot = (int64_t)(idx % (unsigned long long)wq.cap);
    for (int64_t spin = 0;; ++spin) {
        if (__atomic_load_n(&wq.seq[slot], __ATOMIC_ACQUIRE) == idx + 1) break;
        if (ld_acq(&wq.ctr[WQ_ERR]) || spin > SPIN_LIMIT) {
            atomicOr(&wq.ctr[WQ_ERR], 4ull);
            ok = false;
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    ok = true;
    return wq.q[slot];
}

__device__ __forceinline__ void wq_finish(const WorkQ &wq, int cnt) {
    __threadfence();
    if (lane_id() == 0) atomicAdd(&wq.ctr[WQ_DONE], (unsigned long long)cnt);
}

// Row geometry of vertex v: base part then diff part.
struct Row {
    int64_t ob, od;
    int32_t db, tot;
};
__device__ __forceinline__ Row row_of_v(const DirView &g, int32_t v) {
    Row r;
    r.ob = g.off[v];
    r.db = (int32_t)(g.off[v + 1] - r.ob);
    r.od = g.doff[v];
    r.tot = r.db + (int32_t)(g.doff[v + 1] - r.od);
    return r;
}

// Walk the edge ranges [s, s+len) of up to 64 rows (one per lane) with the
// in-wave load-balanced search; fn(valid, owner lane values..., x, w).
template <class Fn>
__device__ __forceinline__ void wave_walk(const DirView &g, int32_t v, int32_t pay, const Row &r, int32_t s,
                                          int32_t len, Fn fn) {
    const int l = lane_id();
    const int64_t incl = wave_incl_scan((int64_t)len);
    const int64_t excl = incl - len;
    const int64_t T = __shfl(incl, WAVE - 1, WAVE);
    for (int64_t eb = 0; eb < T; eb += WAVE) {
        const int64_t e = eb + l;
        int o = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            int cand = o + step;
            int64_t xx = __shfl(excl, cand, WAVE);
            if (xx <= e) o = cand;
        }
        const int32_t vo = __shfl(v, o, WAVE);
        const int32_t po = __shfl(pay, o, WAVE);
        const int64_t obo = __shfl(r.ob, o, WAVE);
        const int64_t odo = __shfl(r.od, o, WAVE);
        const int32_t dbo = __shfl(r.db, o, WAVE);
        const int32_t so = __shfl(s, o, WAVE);
        const int64_t exo = __shfl(excl, o, WAVE);
        bool valid = e < T;
        int32_t x = 0, wt = 0;
        if (valid) {
            int64_t j = so + (e - exo);
            uint32_t c;
            if (j < dbo) { c = (uint32_t)g.col[obo + j]; wt = g.w[obo + j]; }
            else { c = (uint32_t)g.dcol[odo + (j - dbo)]; wt = g.dw[odo + (j - dbo)]; }
            valid = !(c & DEAD);
            x = (int32_t)(c & ID_MASK);
        }
        fn(valid, vo, po, x, wt);
    }
}

// Items of the claimed block: decode, split heavy rows into chunk items, return
// this lane's (v, payload, range).  `whole_hook(v)` runs for whole-row items
// before the row's state is read (SSSP clears the in-queue flag there).
template <class Hook, class Pay>
__device__ __forceinline__ bool wq_items(const WorkQ &wq, const DirView &g, unsigned long long h, int cnt,
                                         int heavy_deg, int chunk, Hook whole_hook, Pay payload, int32_t &v,
                                         int32_t &pay, Row &r, int32_t &s, int32_t &len) {
    const int l = lane_id();
    v = -1;
    pay = 0;
    s = 0;
    len = 0;
    r = Row{0, 0, 0, 0};
    bool ok = true;
    int32_t nch = 0;
    if (l < cnt) {
        int64_t it = wq_read(wq, h + l, ok);
        if (ok) {
            v = (int32_t)(it >> 32);
            uint32_t c = (uint32_t)(it & 0xffffffff);
            if (c == WHOLE) whole_hook(v);
            r = row_of_v(g, v);
            bool live = payload(v, pay);
            if (!live) {
                len = 0;
            } else if (c == WHOLE) {
                if (r.tot > heavy_deg) nch = (r.tot + chunk - 1) / chunk;
                else len = r.tot;
            } else {
                s = (int32_t)c * chunk;
                len = max(0, min(r.tot, s + chunk) - s);
            }
        }
    }
    // hubs: re-enqueue as chunk items
    int32_t mx = wave_max_i32(nch);
    for (int32_t c = 0; c < mx; ++c) wq_push(wq, c < nch, ((int64_t)v << 32) | (uint32_t)c);
    return ballot(!ok) == 0;
}

// ---- SSSP push (Incremental) ------------------------------------------------------

// Per-wave tallies, added to the counters once when the wave leaves.
__device__ __forceinline__ void wq_tally(const WorkQ &wq, int64_t edges, int64_t items) {
    edges = wave_sum(edges);
    items = wave_sum(items);
    if (lane_id() == 0) {
        atomicAdd(&wq.ctr[WT_EDGES], (unsigned long long)edges);
        atomicAdd(&wq.ctr[WT_ITEMS], (unsigned long long)items);
    }
}

__global__ __launch_bounds__(256) void k_wl_push(WorkQ wq, DirView g, uint64_t *key, int32_t *inq, int heavy_deg,
                                                 int chunk) {
    unsigned long long h;
    int cnt;
    int64_t ne = 0, ni = 0;
    while (wq_claim(wq, h, cnt)) {
        if (lane_id() == 0) ni += cnt;
        int32_t v, d;
        Row r;
        int32_t s, len;
        auto hook = [&](int32_t u) {
            atomicExch(&inq[u], 0);
            __threadfence();
        };
        auto pay = [&](int32_t u, int32_t &p) {
            p = sssp_dist(__atomic_load_n(&key[u], __ATOMIC_RELAXED));
            return p < INF;
        };
        bool ok = wq_items(wq, g, h, cnt, heavy_deg, chunk, hook, pay, v, d, r, s, len);
        if (ok) {
            wave_walk(g, v, d, r, s, len, [&](bool valid, int32_t vo, int32_t dov, int32_t x, int32_t w) {
                bool push = false;
                ne += valid;
                if (valid) {
                    uint64_t cand = sssp_pack(dov + w, vo);
                    if (cand < __atomic_load_n(&key[x], __ATOMIC_RELAXED)) {
                        uint64_t old = atomicMin((unsigned long long *)&key[x], (unsigned long long)cand);
                        if (cand < old && sssp_dist(cand) < sssp_dist(old)) push = atomicExch(&inq[x], 1) == 0;
                    }
                }
                wq_push(wq, push, ((int64_t)x << 32) | WHOLE);
            });
        }
        wq_finish(wq, cnt);
    }
    wq_tally(wq, ne, ni);
}

// ---- SSSP subtree cut (Decremental, phase 1) ----------------------------------------
// Every cut vertex is also appended to `list` (for the pull that follows).

__global__ __launch_bounds__(256) void k_wl_cut(WorkQ wq, DirView g, uint64_t *key, int32_t *list,
                                                int heavy_deg, int chunk) {
    unsigned long long h;
    int cnt;
    int64_t ne = 0, ni = 0;
    while (wq_claim(wq, h, cnt)) {
        if (lane_id() == 0) ni += cnt;
        int32_t v, p0;
        Row r;
        int32_t s, len;
        auto hook = [&](int32_t) {};
        auto pay = [&](int32_t, int32_t &p) {
            p = 0;
            return true;
        };
        bool ok = wq_items(wq, g, h, cnt, heavy_deg, chunk, hook, pay, v, p0, r, s, len);
        if (ok) {
            wave_walk(g, v, p0, r, s, len, [&](bool valid, int32_t vo, int32_t, int32_t x, int32_t) {
                bool cut = false;
                ne += valid;
                if (valid && sssp_parent(key[x]) == vo) {
                    key[x] = sssp_pack(INF, -1);
                    cut = true;
                }
                wq_push(wq, cut, ((int64_t)x << 32) | WHOLE);
                int64_t slot = wave_append((int64_t *)&wq.ctr[WQ_LIST], cut);
                if (cut) list[slot] = x;
            });
        }
        wq_finish(wq, cnt);
    }
    wq_tally(wq, ne, ni);
}

// ---- seeding kernels ---------------------------------------------------------------------

__global__ void k_wq_reset(unsigned long long *ctr, int n) {
    if ((int)threadIdx.x < n) ctr[threadIdx.x] = 0;
}

__global__ void k_wq_copy_ctr(unsigned long long *dst, const unsigned long long *src) {
    if (threadIdx.x == 0) *dst = *src;
}

__global__ void k_wq_clear_tags(uint64_t *seq, int64_t cap) {
    for (int64_t i = gtid(); i < cap; i += gstride()) seq[i] = 0;
}

// Enqueue list[0..*count) as whole-row items (cut seeds); also copy them to the
// head of the cut list.
__global__ void k_wl_seed_list(WorkQ wq, const int32_t *seeds, const int64_t *count, int32_t *list) {
    const int64_t nsd = *count;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nsd; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = i < nsd;
        int32_t v = p ? seeds[i] : 0;
        wq_push(wq, p, ((int64_t)v << 32) | WHOLE);
        int64_t slot = wave_append((int64_t *)&wq.ctr[WQ_LIST], p);
        if (p) list[slot] = v;
    }
}

// Cut vertices with a finite pulled distance start the push.
__global__ void k_wl_seed_pulled(WorkQ wq, const int32_t *list, const unsigned long long *count,
                                 const uint64_t *key, int32_t *inq) {
    const int64_t nl = (int64_t)*count;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nl; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < nl) {
            v = list[i];
            p = sssp_dist(key[v]) < INF && atomicExch(&inq[v], 1) == 0;
        }
        wq_push(wq, p, ((int64_t)v << 32) | WHOLE);
    }
}

// OnAdd: inserted arcs relax their heads; improved heads start the push.
__global__ void k_wl_seed_inserts(WorkQ wq, const int64_t *na_p, int64_t na_host, const int32_t *aiu,
                                  const int32_t *aiv, const int32_t *aiw, uint64_t *key, int32_t *inq) {
    const int64_t na = na_p ? *na_p : na_host;
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
                if (cand < old && sssp_dist(cand) < sssp_dist(old)) p = atomicExch(&inq[v], 1) == 0;
            }
        }
        wq_push(wq, p, ((int64_t)v << 32) | WHOLE);
    }
}

// Sources of a (multi-source) static solve.
__global__ void k_wl_seed_sources(WorkQ wq, const int32_t *src, int64_t ns, int32_t *inq) {
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ns; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = i < ns && atomicExch(&inq[src[i]], 1) == 0;
        wq_push(wq, p, ((int64_t)(p ? src[i] : 0) << 32) | WHOLE);
    }
}

// PullOp of sssp.hip, reproduced here so both drivers can use it.
struct WlPullOp {
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

// ---- host side ---------------------------------------------------------------------------

static inline int gridc(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

int wl_groups(dg_graph *g) { return g->cfg.persistent_groups > 0 ? g->cfg.persistent_groups : 1024; }
static int heavy_of(dg_graph *g) { return g->cfg.heavy_degree > 0 ? g->cfg.heavy_degree : 512; }

// Queue storage, counters and in-queue flags for this graph.
static int wl_ensure(dg_graph *g, WorkQ *wq) {
    Work &ws = g->ws;
    int64_t edges = std::max(g->fwd.m + g->fwd.dm, g->rev->m + g->rev->dm);
    int64_t cap = (int64_t)g->n + 2 * (edges / heavy_of(g) + 2) + 64ll * 4 * wl_groups(g) + 4096;
    DG_TRY(ws.wq.ensure((size_t)cap));
    DG_TRY(ws.wseq.ensure((size_t)cap));
    DG_TRY(ws.wctr.ensure(WQ_NCTR * 2));
    if (!ws.inq.p || ws.inq.cap < (size_t)g->n + 1) {
        DG_TRY(ws.inq.ensure((size_t)g->n + 1));
        DG_TRY(fill_i32(ws.inq.p, 0, g->n + 1, g->stream));
    }
    wq->q = ws.wq.p;
    wq->seq = ws.wseq.p;
    wq->cap = (int64_t)std::min(ws.wq.cap, ws.wseq.cap);
    wq->margin = 64ll * 4 * wl_groups(g) + 1024;
    wq->ctr = reinterpret_cast<unsigned long long *>(ws.wctr.p);
    // FIFO relaxation on high-diameter graphs can re-relax each vertex ~sqrt(n)
    // times (static solves refuse such graphs up front); past 4 items per vertex
    // and arc a run stops with an error instead, a fraction of a second of work
    wq->budget = 4ull * (unsigned long long)(g->n + edges) + (1ull << 20);
    return DG_OK;
}

// Fresh queue: counters to zero and every slot's sequence tag to 0.
static int wl_reset(dg_graph *g, const WorkQ &wq) {
    hipLaunchKernelGGL(k_wq_reset, dim3(1), dim3(64), 0, g->stream, wq.ctr, WQ_NCTR);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

static int wl_reset_tally(dg_graph *g, const WorkQ &wq) {
    hipLaunchKernelGGL(k_wq_reset, dim3(1), dim3(64), 0, g->stream, wq.ctr + WT_EDGES, 2);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

// t[0] cut-list length, t[1] arcs examined, t[2] items processed (synchronous).
static int wl_tally(dg_graph *g, const WorkQ &wq, int64_t *t) {
    unsigned long long h[WT_N];
    DG_HIP(hipMemcpyAsync(h, wq.ctr + WT_LIST, sizeof(h), hipMemcpyDeviceToHost, g->stream));
    DG_HIP(hipStreamSynchronize(g->stream));
    for (int i = 0; i < WT_N; ++i) t[i] = (int64_t)h[i];
    return DG_OK;
}

// Algorithmic bytes of the cut and push kernels: per item its queue slot and tag
// (16 B read, 16 B written when it was pushed), the base and diff offset pairs
// (32 B), its key (8 B) and in-queue flag (4 B); per arc the column and weight
// (8 B) and the head's key (8 B).
static double wl_bytes(int64_t edges, int64_t items) { return 16.0 * (double)edges + 76.0 * (double)items; }

static int wl_check(dg_graph *g, const WorkQ &wq, int64_t *list_count) {
    unsigned long long h[WQ_NCTR];
    DG_HIP(hipMemcpyAsync(h, wq.ctr, sizeof(h), hipMemcpyDeviceToHost, g->stream));
    DG_HIP(hipStreamSynchronize(g->stream));
    if (h[WQ_ERR] & 8)
        return set_error(DG_EDEVICE, "work queue passed its work bound (high-diameter graph: use the frontier "
                                     "schedule with near-far buckets, sssp_persistent = 0, sssp_delta > 0)");
    if (h[WQ_ERR]) return set_error(DG_EDEVICE, "work queue error %llu (capacity or wait limit)", h[WQ_ERR]);
    if (list_count) *list_count = (int64_t)h[WQ_LIST];
    return DG_OK;
}

// The sequence tags must never match a future index: clearing them once per
// queue allocation is enough because indices only grow within a run and every run
// starts from index 0 again -- so tags are cleared before every run instead.
static int wl_clear_tags(dg_graph *g, const WorkQ &wq) {
    hipLaunchKernelGGL(k_wq_clear_tags, dim3(gridc(wq.cap)), dim3(256), 0, g->stream, wq.seq, wq.cap);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

int sssp_static_persistent(dg_graph *g, uint64_t *key, const int32_t *sources, int64_t ns) {
    WorkQ wq;
    DG_TRY(wl_ensure(g, &wq));
    hipStream_t s = g->stream;
    DG_TRY(wl_reset(g, wq));
    DG_TRY(wl_reset_tally(g, wq));
    DG_TRY(wl_clear_tags(g, wq));
    hipLaunchKernelGGL(k_wl_seed_sources, dim3(gridc(ns)), dim3(256), 0, s, wq, sources, ns, g->ws.inq.p);
    int ps = prof_begin("sssp_worklist", s);
    hipLaunchKernelGGL(k_wl_push, dim3(wl_groups(g)), dim3(256), 0, s, wq, view(g->fwd), key, g->ws.inq.p,
                       heavy_of(g), heavy_of(g));
    prof_end(ps, s, 0.0);
    DG_HIP(hipGetLastError());
    DG_TRY(wl_check(g, wq, nullptr));
    int64_t t[WT_N];
    DG_TRY(wl_tally(g, wq, t));
    prof_add(ps, wl_bytes(t[1], t[2]));
    return DG_OK;
}

// Dynamic SSSP post-hook on the worklists: enqueue only, no host round trip and
// no allocation, so the sequence can be captured into a hipGraph.  seeds and
// *nseeds_dev: the cut seeds of the pre-hook; cut: output list of every cut
// vertex (capacity n); inserted arcs ws.aiu/aiv/aiw with their count at *ains_dev.
// wl_prepare must have run first (it allocates).
int wl_prepare(dg_graph *g) {
    WorkQ wq;
    DG_TRY(wl_ensure(g, &wq));
    return DG_OK;
}

static int sssp_post_enqueue(dg_graph *g, uint64_t *key, const int32_t *seeds, const int64_t *nseeds_dev,
                             int32_t *cut, const int64_t *ains_dev) {
    WorkQ wq;
    DG_TRY(wl_ensure(g, &wq));
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int H = heavy_of(g);
    // 1. cut the subtrees below the seeds
    DG_TRY(wl_reset(g, wq));
    DG_TRY(wl_reset_tally(g, wq));
    DG_TRY(wl_clear_tags(g, wq));
    hipLaunchKernelGGL(k_wl_seed_list, dim3(64), dim3(256), 0, s, wq, seeds, nseeds_dev, cut);
    hipLaunchKernelGGL(k_wl_cut, dim3(wl_groups(g)), dim3(256), 0, s, wq, view(g->fwd), key, cut, H, H);
    DG_HIP(hipGetLastError());
    // 2. pull once at every cut vertex (count read on the device)
    {
        ExpandArgs a;
        a.F = cut;
        a.nf = 0;
        a.nfp = reinterpret_cast<const int64_t *>(&wq.ctr[WQ_LIST]);
        a.g = view(*g->rev);
        a.hq = reinterpret_cast<int64_t *>(ws.heavy.p);
        a.hcount = ws.dcnt + C_HEAVY;
        a.heavy_deg = H;
        a.chunk = H;
        DG_TRY(counters_clear(g));
        WlPullOp op{key};
        DG_TRY(launch_expand(s, a, op, 4096));
    }
    // 3. push from the pulled cut vertices and the improved heads of inserted arcs
    unsigned long long *listc = wq.ctr + WT_LIST;  // keep the cut count across the reset
    hipLaunchKernelGGL(k_wq_copy_ctr, dim3(1), dim3(64), 0, s, listc, &wq.ctr[WQ_LIST]);
    DG_TRY(wl_reset(g, wq));
    DG_TRY(wl_clear_tags(g, wq));
    hipLaunchKernelGGL(k_wl_seed_pulled, dim3(256), dim3(256), 0, s, wq, cut, listc, key, ws.inq.p);
    hipLaunchKernelGGL(k_wl_seed_inserts, dim3(1024), dim3(256), 0, s, wq, ains_dev, (int64_t)0, ws.aiu.p,
                       ws.aiv.p, ws.aiw.p, key, ws.inq.p);
    hipLaunchKernelGGL(k_wl_push, dim3(wl_groups(g)), dim3(256), 0, s, wq, view(g->fwd), key, ws.inq.p, H, H);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

static int sssp_post_finish(dg_graph *g, int ps, int64_t *ncut_out, int64_t *edges_out) {
    WorkQ wq;
    DG_TRY(wl_ensure(g, &wq));
    DG_TRY(wl_check(g, wq, nullptr));
    int64_t t[WT_N];
    DG_TRY(wl_tally(g, wq, t));
    if (ncut_out) *ncut_out = t[0];
    if (edges_out) *edges_out = t[1];
    prof_add(ps, wl_bytes(t[1], t[2]));
    return DG_OK;
}

int sssp_post_persistent(dg_graph *g, uint64_t *key, const int32_t *seeds, const int64_t *nseeds_dev,
                         int32_t *cut, const int64_t *ains_dev, int64_t *ncut_out, int64_t *edges_out) {
    int ps = prof_begin("sssp_worklist", g->stream);
    DG_TRY(sssp_post_enqueue(g, key, seeds, nseeds_dev, cut, ains_dev));
    prof_end(ps, g->stream, 0.0);
    return sssp_post_finish(g, ps, ncut_out, edges_out);
}

// Same work replayed from a captured hipGraph.  The graph bakes pointers in, so it
// is cached under the set of pointers it uses (the diff level alternates between
// two buffers, so two graphs cover steady state); a new layout captures again.
int graph_replay(dg_graph *g, GraphCache *cache, const std::vector<const void *> &sig,
                 const std::function<int()> &enqueue) {
    if (!g->stream) return set_error(DG_ESTATE, "graph capture needs a non-null stream");
    hipGraphExec_t exec = nullptr;
    for (auto &e : cache->entries)
        if (e.sig == sig) exec = e.exec;
    if (!exec) {
        hipGraph_t graph = nullptr;
        DG_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
        int rc = enqueue();
        hipError_t e = hipStreamEndCapture(g->stream, &graph);
        if (rc != DG_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return set_error(DG_EDEVICE, "stream capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return set_error(DG_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        if (cache->entries.size() >= 16) {
            (void)hipGraphExecDestroy(cache->entries.front().exec);
            cache->entries.erase(cache->entries.begin());
        }
        cache->entries.push_back({sig, exec});
        cache->captures += 1;
    }
    DG_HIP(hipGraphLaunch(exec, g->stream));
    cache->launches += 1;
    return DG_OK;
}

// Same work replayed from a captured hipGraph.  The graph bakes pointers in, so it
// is cached under the set of pointers it uses (the diff level alternates between
// two buffers, so two graphs cover steady state); a new layout captures again.
int sssp_post_graph(dg_graph *g, GraphCache *cache, uint64_t *key, const int32_t *seeds,
                    const int64_t *nseeds_dev, int32_t *cut, const int64_t *ains_dev, int64_t *ncut_out,
                    int64_t *edges_out) {
    DG_TRY(wl_prepare(g));
    std::vector<const void *> sig = {"wl", key, seeds, nseeds_dev, cut, ains_dev, g->fwd.off.p, g->fwd.col.p,
                                     g->fwd.w.p, g->fwd.doff.p, g->fwd.dcol.p, g->fwd.dw.p, g->rev->off.p,
                                     g->rev->col.p, g->rev->w.p, g->rev->doff.p, g->rev->dcol.p, g->rev->dw.p,
                                     g->ws.wq.p, g->ws.wseq.p, g->ws.wctr.p, g->ws.inq.p, g->ws.heavy.p,
                                     g->ws.dcnt, g->ws.aiu.p, g->ws.aiv.p, g->ws.aiw.p};
    sig.push_back(reinterpret_cast<const void *>((intptr_t)g->cfg.heavy_degree));
    sig.push_back(reinterpret_cast<const void *>((intptr_t)g->cfg.persistent_groups));
    int ps = prof_begin("sssp_worklist", g->stream);
    DG_TRY(graph_replay(g, cache, sig, [&]() { return sssp_post_enqueue(g, key, seeds, nseeds_dev, cut, ains_dev); }));
    prof_end(ps, g->stream, 0.0);
    return sssp_post_finish(g, ps, ncut_out, edges_out);
}

void graph_cache_clear(GraphCache *cache) {
    for (auto &e : cache->entries) (void)hipGraphExecDestroy(e.exec);
    cache->entries.clear();
}

}  // namespace dg
