// Internal declarations of the MI355X dynamic-graph library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <functional>
#include <vector>

#include "../../include/dg.h"

struct dg_query;

namespace dg {

// ---- entry encoding --------------------------------------------------------------
// A neighbour entry (base CSR `col`, diff `dcol`) holds the neighbour id in bits
// 0..29 and two flags:
//   DEAD (bit 31): tombstone of a deleted edge (the sentinel of Section 3.5);
//   MARK (bit 30): the entry is touched by the batch in flight -- set on edges the
//         batch deletes until the deletion is committed (pre-hooks read the old
//         graph with it), and on edges the batch inserts until the post-hooks are
//         done.  It plays the role of the edge flags of the Dynamic TC listing.
constexpr uint32_t ID_MASK = 0x3FFFFFFFu;
constexpr uint32_t MARK = 0x40000000u;
constexpr uint32_t DEAD = 0x80000000u;
constexpr int32_t INF = DG_INF;
constexpr int TILE = 256;   // base entries per tombstone counter block (ttomb)

// ---- errors ------------------------------------------------------------------------
int set_error(int code, const char *fmt, ...);
#define DG_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::dg::set_error(DG_EDEVICE, "%s failed: %s (%s:%d)", #expr,         \
                                   hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)
#define DG_TRY(expr)                      \
    do {                                  \
        int r_ = (expr);                  \
        if (r_ != DG_OK) return r_;       \
    } while (0)

// ---- device memory -------------------------------------------------------------------
void *dmalloc(size_t bytes);
void dfree(void *p);

// Growable device buffer.  ensure() keeps contents only when asked.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;
    int ensure(size_t n, bool keep = false, hipStream_t s = nullptr) {
        if (n <= cap && p) return DG_OK;
        size_t nc = n < 64 ? 64 : n + n / 8;
        T *q = static_cast<T *>(dmalloc(nc * sizeof(T)));
        if (!q) return set_error(DG_ENOMEM, "device allocation of %zu bytes failed", nc * sizeof(T));
        if (keep && p && cap) {
            hipError_t e = hipMemcpyAsync(q, p, cap * sizeof(T), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { dfree(q); return set_error(DG_EDEVICE, "copy failed"); }
            (void)hipStreamSynchronize(s);
        }
        release();
        p = q;
        cap = nc;
        return DG_OK;
    }
    void release() {
        if (p) dfree(p);
        p = nullptr;
        cap = 0;
    }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
    }
};

// One direction of the graph store: rows are sources (forward) or destinations
// (reverse).  Base CSR with tombstones plus one sorted diff level (Section 3.5).
struct Dir {
    int32_t n = 0;
    int keybits = 1;          // diff key = (row << keybits) | col
    DBuf<int64_t> off;        // [n+1] base row offsets
    DBuf<int32_t> col, w;     // base entries (DEAD / MARK flags in col)
    int64_t m = 0;            // base entries, tombstones included
    DBuf<int64_t> doff;       // [n+1] diff row offsets
    DBuf<uint64_t> dkey;      // [dm] sorted diff keys
    DBuf<int32_t> dcol, dw;   // [dm] diff entries (flags in dcol)
    int64_t dm = 0;           // diff entries, tombstones included
    DBuf<int32_t> deg;        // [n] live degree
    DBuf<int32_t> ntomb;      // [n] base tombstones per row
    DBuf<int32_t> ttomb;      // [ceil(m/TILE)] base tombstones per merge tile
    int64_t tomb_base = 0;    // host mirrors
    int64_t tomb_diff = 0;
    // spares used by merges and diff rebuilds
    DBuf<int64_t> off2;
    DBuf<int32_t> col2, w2;
    DBuf<uint64_t> dkey2;
    DBuf<int32_t> dcol2, dw2;
};

// Workspace of the radix sort and the scan (sort.hip): one device pool holding
// look-back status words, digit counts and the sort's ping-pong keys and values.
struct SortWork {
    DBuf<uint8_t> pool;
    uint32_t epoch = 0;         // look-back generation of the last pass or scan
    int64_t status_words = 0;   // status words the pool's layout reserves
    int64_t key_cap = 0;        // keys the pool's layout reserves
    uint64_t calls = 0;         // sorts so far: picks which of two digit-count sets a sort uses
    void release() {
        pool.release();
        epoch = 0;
        calls = 0;
        status_words = 0;
        key_cap = 0;
    }
};

// Workspace: scratch grown on demand, reused across batches.
struct Work {
    DBuf<int32_t> bsrc, bdst, bw;
    DBuf<uint8_t> bop;
    DBuf<uint64_t> ikey, ikey_s, rkey, rkey_s;
    DBuf<int32_t> iw, iw_s, rw, rw_s;
    DBuf<int32_t> ddu, ddv;               // deletion arcs to look up
    DBuf<int32_t> adu, adv;               // applied deletion arcs (forward)
    DBuf<int64_t> adpos;                  // position: >= 0 base, < 0 diff (-1 - p)
    DBuf<int32_t> aiu, aiv, aiw;          // applied insertion arcs (forward)
    DBuf<int64_t> aipos;                  // revive position or NEW
    DBuf<uint64_t> nkey;                  // NEW forward keys (sorted)
    DBuf<int32_t> nw;
    DBuf<int32_t> tcu, tcv;               // undirected edges for TC (deleted / inserted)
    DBuf<int64_t> vslot, vpos;            // hole reuse: slot taken per NEW key (+ diff flags), their scan
    DBuf<uint64_t> vkey;                  // hole reuse: NEW keys left for the diff level
    DBuf<int32_t> vw;
    DBuf<int64_t> tcitems;                // TC delta: work items per changed edge, then their scan
    SortWork sw;                          // radix sort / scan workspace (sort.hip)
    DBuf<int64_t> scan64;                 // merge scans
    DBuf<int64_t> tscan;
    // frontier machinery shared by the traversals
    DBuf<int32_t> f0, f1, heavy;          // frontiers and heavy-chunk queue
    DBuf<int32_t> stamp;                  // per-vertex dedup stamps
    DBuf<int32_t> farflag, far0, far1;    // near-far SSSP: far-pile membership stamps and piles
    DBuf<int32_t> nfout;                  // captured near-far rounds: the relaxation's output before the split
    DBuf<int64_t> bpart;                  // per-block partial counts (summed in block order)
    // kept between calls (device frees synchronise the whole device): result
    // staging for host reads and the state of the static comparators
    DBuf<double> rbuf;                    // n + 1 doubles (or 2n + 2 int32)
    DBuf<uint64_t> skey;
    DBuf<double> sx, sc, sxn;
    int32_t far_ctr = 0;
    int32_t stamp_ctr = 0;
    int32_t pr_moves = 0;                 // extrapolation moves of the last PageRank iteration
    DBuf<double> part;                    // partial sums of split rows
    DBuf<double> prs;                     // PageRank scalars: step, dangling mass, constant term
    DBuf<float> prstep;                   // previous PageRank step vector (extrapolated steps' fits)
    DBuf<float> prstep2;                  // the step vector before it (two-step fits)
    DBuf<int32_t> mp_row;                 // merge-path tile starts (row, entry) of the whole-graph pull
    DBuf<int64_t> mp_edge;
    DBuf<double> mp_part;                 // per-tile partial sums of rows split across tiles
    DBuf<int64_t> mp_doff;                // merge tiles: diff-level bounds of each tile's first row
    // device work queue of the persistent traversals (worklist.hip)
    DBuf<int64_t> wq;
    DBuf<uint64_t> wseq, wctr;
    DBuf<int32_t> inq;                    // per-vertex in-queue flags (all zero between runs)
    // counters: device block + pinned host mirror
    int64_t *dcnt = nullptr;
    int64_t *hcnt = nullptr;
    // a merge on the second stream keeps its own error counter and scan scratch
    int64_t *dcnt_m = nullptr;
    int64_t *hcnt_m = nullptr;
    SortWork sw_m;
    hipEvent_t ev[16] = {};
    hipEvent_t step_ev[8] = {};  // completion of the last PageRank steps queued (ring)
};

// Captured hipGraphs of a launch sequence, keyed by the pointers they bake in.
struct GraphCacheEntry {
    std::vector<const void *> sig;
    hipGraphExec_t exec;
};
struct GraphCache {
    std::vector<GraphCacheEntry> entries;
    int64_t captures = 0, launches = 0;
};

enum Counter {
    C_ERR = 0, C_NDEL, C_NINS, C_ADEL, C_IGNDEL, C_DISTINCT, C_AINS, C_IGNINS, C_NEW,
    C_TCDEL, C_TCINS, C_F0, C_F1, C_HEAVY, C_AUX0, C_AUX1, C_AUX2, C_AUX3,
    C_TC0, C_TC1, C_RED0 = 24,
    C_EDGES = 30,  // adjacency entries examined by an SSSP step (base + diff, tombstones included)
    // an upper bound on the longest row (base + diff entries, tombstones included) of
    // either direction: set at build, raised by the rows that gain diff entries, never
    // cleared by counters_clear (the host copy refreshes with every counters_read)
    C_MAXROW = 38,
    // set by a sort or scan whose look-back hit its spin limit; counters_clear
    // leaves it alone, counters_read reports it
    C_SORT_ERR = 39, C_COUNT = 40
};

}  // namespace dg

// ---- handles -------------------------------------------------------------------------
struct dg_graph {
    int32_t n = 0;
    bool undirected = false;
    bool broken = false;
    dg::Dir fwd, rev_own;
    dg::Dir *rev = nullptr;  // == &fwd for undirected graphs
    int64_t m_live = 0;      // live arcs in fwd
    int32_t since_merge = 0; // batches applied since the last merge
    hipStream_t stream = nullptr;
    // while SSSP work runs beside the PageRank steps: called whenever the host waits
    // on the SSSP stream, to keep the PageRank stream queued (null otherwise)
    std::function<void()> *pump = nullptr;
    // vertex order (cfg.vertex_order 0): internal id = perm[caller's id], caller's
    // id = iperm[internal id]; empty when the ids are kept as given
    dg::DBuf<int32_t> perm, iperm;
    bool relabeled = false;
    hipStream_t aux = nullptr;                      // second stream: SSSP beside the PageRank steps
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    dg_config cfg{};
    dg::Work ws;
    std::vector<dg_query *> queries;
};

enum QueryKind { Q_SSSP = 1, Q_PR = 2, Q_TC = 3 };

struct dg_query {
    dg_graph *g = nullptr;
    QueryKind kind = Q_SSSP;
    // SSSP: packed (dist << 32 | parent) keys, parent stored as uint32 (-1 = none)
    int32_t source = 0;
    dg::DBuf<uint64_t> key;
    dg::DBuf<int32_t> inval;  // cut vertices (seeds first)
    int64_t nseeds = 0;
    dg::DBuf<int64_t> qcnt;   // device copies of nseeds and the applied-insert count
    int64_t *hpin = nullptr;  // pinned staging for qcnt
    dg::DBuf<int32_t> srcs;   // device list of sources (multi-source: one per member graph)
    int64_t nsrc = 0;         // 0: single source `source`
    dg::GraphCache *gcache = nullptr;  // replay the update from captured hipGraphs (owned by a set, or own_cache)
    dg::GraphCache *own_cache = nullptr;
    dg::DBuf<int32_t> gstamp;  // dedup stamps of the captured frontier rounds (device-side stamp counter)
    dg::DBuf<int32_t> gfar;    // far-pile membership stamps of the captured near-far rounds
    // PageRank: unnormalised x of the dangling-dropped system, x/outdeg cache
    double damping = 0.85, tol = 1e-9;
    int32_t max_iter = 1000;
    dg::DBuf<double> x, xn, contrib;
    dg::DBuf<double> res;     // residual of every vertex (residual push, cfg.pr_mode 3)
    int32_t last_iters = 0;
    int32_t converged = 0;
    // triangle count
    uint64_t tc = 0;
};

struct dg_snapshot {
    dg_graph *g = nullptr;
    std::vector<std::pair<void *, size_t>> bufs;  // device copies in a fixed order
    std::vector<int64_t> scalars;
    std::vector<dg_query *> queries;
};

namespace dg {
// graph store (graph.hip)
int graph_build(dg_graph *g, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *w);
int graph_export(dg_graph *g, int64_t *m, int32_t *src, int32_t *dst, int32_t *w);
int graph_merge(dg_graph *g);
// expect_op >= 0: every op must equal it (partially dynamic modes), else DG_EINVAL.
int apply_chunk(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst, const int32_t *w,
                const uint8_t *op, bool dev, dg_batch_stats *st, int expect_op = -1);
int counters_read(dg_graph *g);
int counters_clear(dg_graph *g);
int ws_init(dg_graph *g);
void ws_free(dg_graph *g);
void dir_free(Dir &d);
int next_stamp(dg_graph *g, int32_t *stamp);
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
int scan_excl(dg_graph *g, const int64_t *in, int64_t *out, int64_t n);  // exclusive prefix sum

// sort.hip: stable LSD radix sort of (key, value) pairs on the low `bits` bits of
// the keys (kin/vin are not modified; kout/vout must not alias them), and an
// exclusive scan of non-negative int64 values (total below 2^48).  On a look-back
// spin-limit exit they OR a bit into *err (device memory).
int radix_sort_pairs(hipStream_t s, SortWork &w, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                     int32_t *vout, int64_t n, int bits, int64_t *err);
int scan_excl_i64(hipStream_t s, SortWork &w, const int64_t *in, int64_t *out, int64_t n, int64_t *err);
int fill_u64_on(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);

// SSSP (sssp.hip)
int sssp_init(dg_query *q);
int sssp_static_solve(dg_graph *g, uint64_t *key, int32_t source, dg_batch_stats *st);
int sssp_pre_delete(dg_query *q, int64_t n_applied_del);
int sssp_post_update(dg_query *q, int64_t n_applied_del, int64_t n_applied_ins, dg_batch_stats *st);
int sssp_read(dg_query *q, int32_t *dist, int32_t *parent, bool dev);
int sssp_unpack(dg_graph *g, const uint64_t *key, int32_t *dist, int32_t *parent, hipStream_t s);
// Checkpoint/resume: keys from host (dist, parent) in the caller's ids, checked
// against the current graph (DG_EINVAL unless they are its shortest paths).
int sssp_import(dg_query *q, const int32_t *dist, const int32_t *parent);

// handles (capi.hip)
int graph_create_dev(int32_t n, int64_t m, const int32_t *ds, const int32_t *dd, const int32_t *dw,
                     const dg_config *cfg, hipStream_t stream, dg_graph **out);
int query_attach(dg_graph *g, dg_query *q, dg_query **out);

// persistent worklist traversals (worklist.hip)
int sssp_static_persistent(dg_graph *g, uint64_t *key, const int32_t *sources, int64_t ns);
// ncut_out: vertices cut; edges_out: arcs examined by the cut and push kernels.
int sssp_post_persistent(dg_graph *g, uint64_t *key, const int32_t *seeds, const int64_t *nseeds_dev,
                         int32_t *cut, const int64_t *ains_dev, int64_t *ncut_out, int64_t *edges_out);
int sssp_post_graph(dg_graph *g, GraphCache *cache, uint64_t *key, const int32_t *seeds,
                    const int64_t *nseeds_dev, int32_t *cut, const int64_t *ains_dev, int64_t *ncut_out,
                    int64_t *edges_out);
void graph_cache_clear(GraphCache *cache);
// Launch the hipGraph cached under `sig`, capturing `enqueue` on g->stream first
// if there is none (enqueue must not allocate or synchronise).
int graph_replay(dg_graph *g, GraphCache *cache, const std::vector<const void *> &sig,
                 const std::function<int()> &enqueue);
int wl_prepare(dg_graph *g);
int wl_groups(dg_graph *g);
int sssp_static_multi(dg_graph *g, uint64_t *key, const int32_t *srcs, int64_t ns, dg_batch_stats *st);

// PageRank (pagerank.hip)
int pr_init(dg_query *q);
int pr_static_solve(dg_graph *g, double damping, double tol, int32_t max_iter, double *x,
                    double *contrib, double *xn, int32_t *iters, int32_t *conv);
// Work run once while PageRank steps are in flight on the graph's stream (or, where
// they cannot overlap it, after them); its return code is kept in rc.
// Wait for stream st.  While SSSP work runs beside the PageRank steps (g->pump
// set), the host polls instead of blocking and keeps queuing the steps between
// polls, so the PageRank stream does not run dry while the host drives the SSSP
// rounds.
inline hipError_t wait_stream(dg_graph *g, hipStream_t st) {
    if (g->pump)
        while (hipStreamQuery(st) == hipErrorNotReady) (*g->pump)();
    return hipStreamSynchronize(st);
}

struct SideWork {
    std::function<int()> fn;
    bool beside = false;  // set when it runs while the steps are in flight
    bool done = false;
    int rc = DG_OK;
    void run() {
        if (!done) {
            done = true;
            rc = fn();
        }
    }
};
// side (nullable) runs exactly once: right after the first group of whole-graph
// tile steps is enqueued, else after the update.
// Internal id of a caller's vertex id (identity when the ids are kept as given).
int vertex_in(dg_graph *g, int32_t v, int32_t *out);
int pr_post_update(dg_query *q, int64_t n_applied_del, int64_t n_applied_ins, dg_batch_stats *st,
                   SideWork *side = nullptr);
int pr_read(dg_query *q, double *rank, bool dev);
int pr_normalize(dg_graph *g, const double *x, double *rank, bool dev);
// Checkpoint/resume: x in the caller's order to and from host memory; an import
// converges from the given values (one step when they are already converged).
int pr_export(dg_query *q, double *x);
// pr_read without any device allocation (fixed per-device scratch array).
int pr_read_noalloc(dg_query *q, double *rank, bool dev);
int pr_gather_floor(dg_graph *g, int32_t reps, double *us);
int pr_import(dg_query *q, const double *x);

// launch timing (prof.hip)
bool prof_on();
int prof_begin(const char *name, hipStream_t s);
void prof_end(int slot, hipStream_t s, double bytes);
// Add bytes to a recorded launch once they are known (after the launch finished).
void prof_add(int slot, double bytes);
// Forget a recorded launch (it did no work).
void prof_drop(int slot);

// triangle counting (tc.hip)
int tc_count_static(dg_graph *g, uint64_t *count);
int tc_delta(dg_graph *g, const int32_t *eu, const int32_t *ev, int64_t ne, uint64_t *sum6,
             int64_t *entries = nullptr);
}  // namespace dg
