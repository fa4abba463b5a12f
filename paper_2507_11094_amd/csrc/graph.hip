// Graph store: build, batch application (updateCSRDel / updateCSRAdd) and merge.
//
// The store is the diff-CSR of Section 3.5 re-laid for MI355X: per direction a
// sorted base CSR whose deleted entries keep their slot with a tombstone bit (the
// paper's sentinel), plus ONE sorted diff level that collects insertions.  Each
// batch merges its insertions into the diff (instead of chaining a new diff per
// batch); when diff entries plus tombstones pass a threshold the diff and the
// tombstones are merged into a fresh base CSR by a coalesced tile-parallel stream
// (Section 3.5: the chain is merged after a configurable number of batches).
#include <algorithm>
#include <cstring>

#include "dg_device.h"

namespace dg {

static int keybits_for(int32_t n) {
    int b = 1;
    while ((1ll << b) < (int64_t)n) ++b;
    return b;
}

static inline int grid_for(int64_t n, int block = 256, int cap = 8192) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Blocks for the chunked kernels (CH elements per block and pass).
static inline int grid_ch(int64_t n) { return grid_for(n, CH, 8192); }

// ---------------------------------------------------------------- small kernels

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DG_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    DG_HIP(hipGetLastError());
    return DG_OK;
}
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DG_OK;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

// ---------------------------------------------------------------- sort and scan (sort.hip)

// Timed as whole calls (all their launches): 8 B read + 8 B written per value of a
// scan, 12 B read + 12 B written per pair of a sort (each pass moves them again).
static int scan_excl_on(hipStream_t s, SortWork &w, int64_t *err, const int64_t *in, int64_t *out, int64_t n) {
    const int ps = prof_begin("scan", s);
    const int rc = scan_excl_i64(s, w, in, out, n, err);
    prof_end(ps, s, 16.0 * (double)n);
    return rc;
}

static int sort_pairs(dg_graph *g, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                      int32_t *vout, int64_t n, int bits) {
    const int ps = prof_begin("sort_pairs", g->stream);
    const int rc = radix_sort_pairs(g->stream, g->ws.sw, kin, kout, vin, vout, n, bits, g->ws.dcnt + C_SORT_ERR);
    prof_end(ps, g->stream, 24.0 * (double)n);
    return rc;
}

int scan_excl(dg_graph *g, const int64_t *in, int64_t *out, int64_t n) {
    return scan_excl_on(g->stream, g->ws.sw, g->ws.dcnt + C_SORT_ERR, in, out, n);
}

// ---------------------------------------------------------------- counters

int counters_clear(dg_graph *g) { return fill_i64(g->ws.dcnt, 0, C_MAXROW, g->stream); }

int counters_read(dg_graph *g) {
    DG_HIP(hipMemcpyAsync(g->ws.hcnt, g->ws.dcnt, sizeof(int64_t) * C_COUNT, hipMemcpyDeviceToHost,
                          g->stream));
    DG_HIP(wait_stream(g, g->stream));
    if (g->ws.hcnt[C_SORT_ERR]) return set_error(DG_EDEVICE, "sort or scan look-back did not finish (internal error)");
    return DG_OK;
}

int ws_init(dg_graph *g) {
    g->ws.dcnt = static_cast<int64_t *>(dmalloc(sizeof(int64_t) * C_COUNT));
    if (!g->ws.dcnt) return set_error(DG_ENOMEM, "counter allocation failed");
    // C_COUNT counter slots, then 8 slots of PageRank step state
    DG_HIP(hipHostMalloc((void **)&g->ws.hcnt, sizeof(int64_t) * (C_COUNT + 16), hipHostMallocDefault));
    g->ws.dcnt_m = static_cast<int64_t *>(dmalloc(sizeof(int64_t) * C_COUNT));
    if (!g->ws.dcnt_m) return set_error(DG_ENOMEM, "counter allocation failed");
    DG_HIP(hipHostMalloc((void **)&g->ws.hcnt_m, sizeof(int64_t) * C_COUNT, hipHostMallocDefault));
    for (auto &e : g->ws.ev) DG_HIP(hipEventCreate(&e));
    DG_TRY(fill_i64(g->ws.dcnt_m, 0, C_COUNT, g->stream));
    return fill_i64(g->ws.dcnt, 0, C_COUNT, g->stream);
}

void dir_free(Dir &d) {
    d.off.release(); d.col.release(); d.w.release(); d.doff.release(); d.dkey.release();
    d.dcol.release(); d.dw.release(); d.deg.release(); d.ntomb.release(); d.ttomb.release();
    d.off2.release(); d.col2.release(); d.w2.release(); d.dkey2.release(); d.dcol2.release();
    d.dw2.release();
}

void ws_free(dg_graph *g) {
    Work &w = g->ws;
    w.bsrc.release(); w.bdst.release(); w.bw.release(); w.bop.release();
    w.ikey.release(); w.ikey_s.release(); w.rkey.release(); w.rkey_s.release();
    w.iw.release(); w.iw_s.release(); w.rw.release(); w.rw_s.release();
    w.ddu.release(); w.ddv.release(); w.adu.release(); w.adv.release(); w.adpos.release();
    w.aiu.release(); w.aiv.release(); w.aiw.release(); w.aipos.release();
    w.nkey.release(); w.nw.release(); w.tcu.release(); w.tcv.release(); w.sw.release();
    w.scan64.release(); w.tscan.release(); w.f0.release(); w.f1.release(); w.heavy.release();
    w.stamp.release(); w.part.release(); w.prs.release();
    w.mp_row.release(); w.mp_edge.release(); w.mp_part.release(); w.mp_doff.release(); w.tcitems.release();
    w.farflag.release(); w.far0.release(); w.far1.release(); w.nfout.release(); w.bpart.release();
    w.prstep.release();
    w.prstep2.release();
    w.rbuf.release(); w.skey.release(); w.sx.release(); w.sc.release(); w.sxn.release();
    w.vslot.release(); w.vpos.release(); w.vkey.release(); w.vw.release();
    w.wq.release(); w.wseq.release(); w.wctr.release(); w.inq.release();
    g->perm.release(); g->iperm.release();
    if (w.dcnt) dfree(w.dcnt);
    if (w.hcnt) (void)hipHostFree(w.hcnt);
    if (w.dcnt_m) dfree(w.dcnt_m);
    if (w.hcnt_m) (void)hipHostFree(w.hcnt_m);
    w.sw_m.release();
    w.dcnt_m = nullptr;
    w.hcnt_m = nullptr;
    if (g->aux) (void)hipStreamDestroy(g->aux);
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    if (g->ev_join) (void)hipEventDestroy(g->ev_join);
    g->aux = nullptr;
    g->ev_fork = g->ev_join = nullptr;
    for (auto &e : w.ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : w.step_ev)
        if (e) (void)hipEventDestroy(e);
    w.dcnt = nullptr;
    w.hcnt = nullptr;
}

// Fresh per-vertex stamp value (stamps dedup frontier pushes without clearing).
int next_stamp(dg_graph *g, int32_t *stamp) {
    Work &w = g->ws;
    if (!w.stamp.p || w.stamp_ctr >= INT32_MAX - 4) {
        DG_TRY(w.stamp.ensure((size_t)g->n + 1));
        DG_TRY(fill_i32(w.stamp.p, 0, g->n + 1, g->stream));
        w.stamp_ctr = 0;
    }
    *stamp = ++w.stamp_ctr;
    return DG_OK;
}

// ---------------------------------------------------------------- build

__global__ void k_validate_edges(int64_t m, const int32_t *s, const int32_t *d, const int32_t *w,
                                 int32_t n, int64_t *cnt) {
    for (int64_t i = gtid(); i < m; i += gstride()) {
        int32_t u = s[i], v = d[i];
        bool bad = u < 0 || u >= n || v < 0 || v >= n || u == v;
        if (w) bad |= (w[i] < 1 || w[i] >= (1 << 30));
        if (bad) atomicOr((unsigned long long *)&cnt[C_ERR], 1ull);
    }
}

__global__ void k_make_keys(int64_t m, const int32_t *s, const int32_t *d, const int32_t *w, int B,
                            int reverse, int both, const int32_t *perm, uint64_t *keys, int32_t *vals) {
    for (int64_t i = gtid(); i < m; i += gstride()) {
        uint32_t u = (uint32_t)s[i], v = (uint32_t)d[i];
        if (perm) {
            u = (uint32_t)perm[u];
            v = (uint32_t)perm[v];
        }
        if (reverse) { uint32_t t = u; u = v; v = t; }
        int32_t wt = w ? w[i] : 1;
        keys[i] = ((uint64_t)u << B) | v;
        vals[i] = wt;
        if (both) {
            keys[m + i] = ((uint64_t)v << B) | u;
            vals[m + i] = wt;
        }
    }
}

__global__ void k_check_dup(int64_t m, const uint64_t *k, int64_t *cnt) {
    for (int64_t i = gtid() + 1; i < m; i += gstride())
        if (k[i] == k[i - 1]) atomicOr((unsigned long long *)&cnt[C_ERR], 2ull);
}

__global__ void k_split_keys(int64_t m, const uint64_t *k, const int32_t *vals, int B, int32_t *col,
                             int32_t *w) {
    const uint64_t mask = (1ull << B) - 1;
    for (int64_t i = gtid(); i < m; i += gstride()) {
        col[i] = (int32_t)(k[i] & mask);
        w[i] = vals[i];
    }
}

// off[r] = first position whose row is >= r, for r in [0, n]
__global__ void k_row_offsets(int32_t n, const uint64_t *k, int64_t m, int B, int64_t *off) {
    for (int64_t r = gtid(); r <= n; r += gstride()) off[r] = lower_key(k, 0, m, (uint64_t)r << B);
}

// Row lengths, and their maximum raised into *maxrow.
__global__ void k_degrees(int32_t n, const int64_t *off, int32_t *deg, int64_t *maxrow) {
    int64_t mx = 0;
    for (int64_t r = gtid(); r < n; r += gstride()) {
        const int64_t len = off[r + 1] - off[r];
        deg[r] = (int32_t)len;
        mx = max(mx, len);
    }
    mx = wave_max(mx);
    if (lane_id() == 0 && mx > 0) atomicMax((unsigned long long *)maxrow, (unsigned long long)mx);
}

// The rows that gained the diff keys k[0, nk): their total lengths (base entries,
// tombstones included, plus diff entries) raised into *maxrow.
__global__ void k_diff_row_max(int64_t nk, const uint64_t *k, int B, const int64_t *off, const int64_t *doff,
                               int64_t *maxrow) {
    int64_t mx = 0;
    for (int64_t j = gtid(); j < nk; j += gstride()) {
        const int32_t r = (int32_t)(k[j] >> B);
        mx = max(mx, (off[r + 1] - off[r]) + (doff[r + 1] - doff[r]));
    }
    mx = wave_max(mx);
    if (lane_id() == 0 && mx > 0) atomicMax((unsigned long long *)maxrow, (unsigned long long)mx);
}

static int64_t ntiles_for(int64_t m) { return (m + TILE - 1) / TILE; }

static int dir_from_sorted(dg_graph *g, Dir &d, const uint64_t *keys, const int32_t *vals, int64_t m,
                           int B) {
    hipStream_t s = g->stream;
    d.n = g->n;
    d.keybits = B;
    d.m = m;
    d.dm = 0;
    d.tomb_base = 0;
    d.tomb_diff = 0;
    DG_TRY(d.off.ensure(g->n + 1));
    DG_TRY(d.col.ensure(m + 1));
    DG_TRY(d.w.ensure(m + 1));
    DG_TRY(d.deg.ensure(g->n + 1));
    DG_TRY(d.ntomb.ensure(g->n + 1));
    DG_TRY(d.ttomb.ensure(ntiles_for(m) + 2));
    DG_TRY(d.doff.ensure(g->n + 1));
    if (m > 0)
        hipLaunchKernelGGL(k_split_keys, dim3(grid_for(m)), dim3(256), 0, s, m, keys, vals, B,
                           d.col.p, d.w.p);
    hipLaunchKernelGGL(k_row_offsets, dim3(grid_for(g->n + 1)), dim3(256), 0, s, g->n, keys, m, B,
                       d.off.p);
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, d.off.p, d.deg.p,
                       g->ws.dcnt + C_MAXROW);
    DG_HIP(hipGetLastError());
    DG_TRY(fill_i32(d.ntomb.p, 0, g->n + 1, s));
    DG_TRY(fill_i32(d.ttomb.p, 0, ntiles_for(m) + 2, s));
    DG_TRY(fill_i64(d.doff.p, 0, g->n + 1, s));
    return DG_OK;
}

// Vertex order by degree: key = (INT32_MAX - degree) above the id, so that an
// ascending sort puts the highest degree first and breaks ties by id.
__global__ void k_order_keys(int32_t n, const int64_t *off, int B, uint64_t *keys, int32_t *vals) {
    for (int64_t v = gtid(); v < n; v += gstride()) {
        const int64_t deg = off[v + 1] - off[v];
        keys[v] = ((uint64_t)(INT32_MAX - (int32_t)min(deg, (int64_t)INT32_MAX)) << B) | (uint64_t)v;
        vals[v] = (int32_t)v;
    }
}

__global__ void k_perm_from_order(int32_t n, const int32_t *order, int32_t *perm, int32_t *iperm) {
    for (int64_t i = gtid(); i < n; i += gstride()) {
        const int32_t v = order[i];
        iperm[i] = v;
        perm[v] = (int32_t)i;
    }
}

// perm / iperm of the degree order of a validated edge list: the out-degree (the
// degree, undirected) of every given id, then a sort of (degree, id).
static int vertex_order_build(dg_graph *g, int64_t m, const int32_t *src, const int32_t *dst, int B) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int32_t n = g->n;
    const int64_t arcs = g->undirected ? 2 * m : m;
    const size_t cap = (size_t)std::max<int64_t>(arcs, n) + 1;
    DG_TRY(ws.ikey.ensure(cap));
    DG_TRY(ws.ikey_s.ensure(cap));
    DG_TRY(ws.iw.ensure(cap));
    DG_TRY(ws.iw_s.ensure(cap));
    DG_TRY(ws.scan64.ensure((size_t)n + 1));
    DG_TRY(g->perm.ensure((size_t)n + 1));
    DG_TRY(g->iperm.ensure((size_t)n + 1));
    if (m > 0)
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(m)), dim3(256), 0, s, m, src, dst, (const int32_t *)nullptr,
                           B, 0, (int)g->undirected, (const int32_t *)nullptr, ws.ikey.p, ws.iw.p);
    DG_HIP(hipGetLastError());
    DG_TRY(sort_pairs(g, ws.ikey.p, ws.ikey_s.p, ws.iw.p, ws.iw_s.p, arcs, 2 * B));
    hipLaunchKernelGGL(k_row_offsets, dim3(grid_for(n + 1)), dim3(256), 0, s, n, ws.ikey_s.p, arcs, B,
                       ws.scan64.p);
    hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n)), dim3(256), 0, s, n, ws.scan64.p, B, ws.ikey.p, ws.iw.p);
    DG_HIP(hipGetLastError());
    DG_TRY(sort_pairs(g, ws.ikey.p, ws.ikey_s.p, ws.iw.p, ws.iw_s.p, n, B + 31));
    hipLaunchKernelGGL(k_perm_from_order, dim3(grid_for(n)), dim3(256), 0, s, n, ws.iw_s.p, g->perm.p,
                       g->iperm.p);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

int vertex_in(dg_graph *g, int32_t v, int32_t *out) {
    if (!g->relabeled) {
        *out = v;
        return DG_OK;
    }
    DG_HIP(hipMemcpyAsync(out, g->perm.p + v, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    DG_HIP(hipStreamSynchronize(g->stream));
    return DG_OK;
}

int graph_build(dg_graph *g, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *w) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int B = keybits_for(g->n);
    DG_TRY(counters_clear(g));
    if (m > 0)
        hipLaunchKernelGGL(k_validate_edges, dim3(grid_for(m)), dim3(256), 0, s, m, src, dst, w, g->n,
                           ws.dcnt);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    if (ws.hcnt[C_ERR]) return set_error(DG_EINVAL, "edge list holds a self-loop, an id outside [0,n) or a weight outside [1,2^30)");
    const int64_t arcs = g->undirected ? 2 * m : m;
    if (arcs > INT32_MAX) return set_error(DG_EINVAL, "more than 2^31 arcs");
    if (g->relabeled) DG_TRY(vertex_order_build(g, m, src, dst, B));
    const int32_t *perm = g->relabeled ? g->perm.p : nullptr;
    DG_TRY(ws.ikey.ensure(arcs + 1));
    DG_TRY(ws.ikey_s.ensure(arcs + 1));
    DG_TRY(ws.iw.ensure(arcs + 1));
    DG_TRY(ws.iw_s.ensure(arcs + 1));
    for (int dir = 0; dir < (g->undirected ? 1 : 2); ++dir) {
        if (m > 0)
            hipLaunchKernelGGL(k_make_keys, dim3(grid_for(m)), dim3(256), 0, s, m, src, dst, w, B, dir,
                               (int)g->undirected, perm, ws.ikey.p, ws.iw.p);
        DG_HIP(hipGetLastError());
        DG_TRY(sort_pairs(g, ws.ikey.p, ws.ikey_s.p, ws.iw.p, ws.iw_s.p, arcs, 2 * B));
        if (dir == 0) {
            if (arcs > 1)
                hipLaunchKernelGGL(k_check_dup, dim3(grid_for(arcs)), dim3(256), 0, s, arcs, ws.ikey_s.p,
                                   ws.dcnt);
            DG_TRY(counters_read(g));
            if (ws.hcnt[C_ERR]) return set_error(DG_EINVAL, "edge list holds a repeated edge");
        }
        Dir &d = dir == 0 ? g->fwd : g->rev_own;
        DG_TRY(dir_from_sorted(g, d, ws.ikey_s.p, ws.iw_s.p, arcs, B));
    }
    g->rev = g->undirected ? &g->fwd : &g->rev_own;
    g->m_live = arcs;
    // the build-sized scratch is not needed again
    ws.ikey.release(); ws.ikey_s.release(); ws.iw.release(); ws.iw_s.release(); ws.sw.release();
    return counters_read(g);  // also brings the longest-row bound to the host
}

// ---------------------------------------------------------------- merge (Section 3.5)

__global__ void k_deg_to_i64(int32_t n, const int32_t *deg, int64_t *out) {
    for (int64_t i = gtid(); i <= n; i += gstride()) out[i] = i < n ? deg[i] : 0;
}

// Merge of one direction on merge-path tiles: the row ends and the base entries
// form one sequence of n + m items and each workgroup takes MG_ITEMS of them, so
// every workgroup moves the same amount whatever the row lengths.  A tile stages
// its rows' starts and diff ranges in LDS, reads its entries once (coalesced), and
// writes each live entry to
//   (entry index) - (tombstones before it) + doff[r] + (diff entries of r below it)
// which is its place in the merged level because the diff level holds live
// entries only when the merge runs.  Tombstones before the entry come from the
// per-block counters (ttomb, TILE entries each, kept by the delete step) plus a
// ballot count inside the tile.  Diff entries are written at their insertion
// points by the base entries of their row (rows with an empty base part:
// k_merge_diff_empty).
constexpr int MG_THREADS = 256;
constexpr int MG_ITEMS = 2048;  // default items per tile (cfg.merge_tile picks 512 / 1024 / 2048)
constexpr int MG_WAVES = MG_THREADS / WAVE;

// Tile b starts at (mp_row[b], mp_edge[b]); mp_dlo[b] = doff[row] and mp_dhi[b] =
// doff[row + 1] (clamped to n) bound the diff entries of its rows without a
// dependent load inside the tile kernel.
__global__ void k_mg_partition(const int64_t *__restrict__ off, const int64_t *__restrict__ doff, int32_t n,
                               int64_t m, int64_t nb, int items, int32_t *mp_row, int64_t *mp_edge,
                               int64_t *mp_dlo, int64_t *mp_dhi) {
    for (int64_t b = gtid(); b <= nb; b += gstride()) {
        const int64_t diag = min(b * (int64_t)items, (int64_t)n + m);
        int64_t lo = max(diag - m, (int64_t)0), hi = min(diag, (int64_t)n);
        while (lo < hi) {
            const int64_t p = (lo + hi) >> 1;
            if (off[p + 1] <= diag - p - 1) lo = p + 1;
            else hi = p;
        }
        mp_row[b] = (int32_t)lo;
        mp_edge[b] = diag - lo;
        mp_dlo[b] = doff[lo];
        mp_dhi[b] = doff[min(lo + 1, (int64_t)n)];
    }
}

__device__ __forceinline__ void merge_put(int32_t *col2, int32_t *w2, int64_t cap, int64_t o, int32_t c,
                                          int32_t wt, int64_t *cnt) {
    if (o >= 0 && o < cap) {
        col2[o] = c;
        w2[o] = wt;
    } else {
        atomicOr((unsigned long long *)&cnt[C_ERR], 4ull);
    }
}


__device__ __forceinline__ int lds_lower(const int32_t *a, int lo, int hi, uint32_t v) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (((uint32_t)a[mid] & ID_MASK) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ITEMS rows + entries per tile; up to min(ITEMS / 4, 256) diff entries (column and
// weight) of its rows are staged in LDS (more are read from memory).  Output
// positions need no per-row output
// offsets: after the update the diff level holds live entries only, so
//   off2[r] = (base entries before row r) - (tombstones before row r) + doff[r],
// and a live base entry i of row r lands at
//   i - (tombstones before i) + doff[r] + (diff entries of row r below it),
// the tombstones before i coming from the per-block counters (TB) and a ballot
// count inside the tile.  A tile keeps about 9 bytes of LDS per item (row starts
// and diff ranges, plus the staged diff entries); the entries stay in
// registers and the column before an entry comes from the neighbouring lane (or
// the wave before).  No global load follows the tile's first barrier except for
// tiles whose diff entries exceed the staging: on this GPU a wave's load counter
// also counts its stores, so a load after the first stores would wait for them.
template <int ITEMS>
__global__ __launch_bounds__(MG_THREADS, 8) void k_merge_tiles(
    int32_t n, const int32_t *__restrict__ mp_row, const int64_t *__restrict__ mp_edge,
    const int64_t *__restrict__ mp_dlo, const int64_t *__restrict__ mp_dhi,
    const int64_t *__restrict__ off, const int32_t *__restrict__ col, const int32_t *__restrict__ w,
    const int64_t *__restrict__ doff, const int32_t *__restrict__ dcol, const int32_t *__restrict__ dw,
    const int64_t *__restrict__ TB, int32_t *__restrict__ col2, int32_t *__restrict__ w2, int64_t cap, uint32_t keep,
    int64_t *cnt) {
    constexpr int IPT = ITEMS / MG_THREADS;
    constexpr int DC = ITEMS / 4 < 256 ? ITEMS / 4 : 256;
    __shared__ int32_t s_off[ITEMS + 1];  // row start - e0 (row 0: -1 when it began earlier)
    __shared__ int32_t s_dlo[ITEMS + 2];  // doff[r] - doff[r0]
    __shared__ int32_t s_dc[DC], s_dw[DC];  // the tile's diff entries
    __shared__ int32_t s_wd[IPT][MG_WAVES];  // tombstones per wave and item round
    __shared__ uint32_t s_last[IPT][MG_WAVES + 1];  // column of each wave's last entry; [0][0]: entry e0 - 1
    __shared__ int64_t s_base[3];          // off[r0], tombstones before e0, off[r1 + 1]
    const int64_t b = blockIdx.x;
    const int32_t r0 = mp_row[b], r1 = mp_row[b + 1];
    const int64_t e0 = mp_edge[b];
    const int32_t ne = (int32_t)(mp_edge[b + 1] - e0);
    const int32_t nr = r1 - r0;
    const int64_t dbase = mp_dlo[b];           // the diff entries of the tile's rows
    const int64_t ndt = mp_dhi[b + 1] - dbase; // (one contiguous range of the diff level)
    const bool dlds = ndt <= DC;
    const int64_t st = (e0 / TILE) * TILE;     // counter block of e0
    const int64_t tb0 = TB[e0 / TILE];
    const int t = threadIdx.x, wv = t / WAVE, l = lane_id();
    // Every load of the tile is issued before the first one is used, so the tile
    // waits for one memory round trip after its partition entry, not one per item.
    uint32_t c[IPT];
    int32_t wt[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int j = u * MG_THREADS + t;
        c[u] = j < ne ? (uint32_t)col[e0 + j] : 0u;
        wt[u] = j < ne ? w[e0 + j] : 0;
    }
    // row r0 + t (slot nr + 1: the end of the row still open at the tile's end)
    const bool has_row = t <= nr + 1 && r0 + t <= n;
    const int64_t ro_t = *(has_row ? off + r0 + t : mp_edge + b);
    const int64_t rd_t = *(has_row ? doff + r0 + t : mp_edge + b);
    // (lanes with nothing to load read the tile's own partition entry instead, so
    // that no load sits behind a branch that would make the wave wait on it)
    const bool has_dc = dlds && t < ndt;
    const int32_t dc_raw = *(has_dc ? dcol + dbase + t : mp_row + b);
    const int32_t dw_raw = *(has_dc ? dw + dbase + t : mp_row + b);
    const int32_t prev_raw = *(t == 0 && e0 > 0 ? col + e0 - 1 : mp_row + b);
    // wave 0: the entries of e0's counter block before e0
    uint32_t tbc[TILE / WAVE];
#pragma unroll
    for (int q = 0; q < TILE / WAVE; ++q) {
        const int64_t idx = st + q * WAVE + l;
        tbc[q] = (uint32_t) * (wv == 0 && idx < e0 ? col + idx : mp_row + b);
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const uint64_t bm = ballot((c[u] & DEAD) != 0u);
        if (l == 0) s_wd[u][wv] = __popcll(bm);
        if (l == WAVE - 1) s_last[u][wv + 1] = c[u];
    }
    if (t == 0) s_last[0][0] = (uint32_t)prev_raw;
    auto put_row = [&](int i, int64_t ro, int64_t rd) {
        if (r0 + i > n) return;
        s_dlo[i] = (int32_t)(rd - dbase);
        if (i <= nr) {
            const int64_t o = ro - e0;
            s_off[i] = (int32_t)(o < 0 ? -1 : o);
        } else {
            s_base[2] = ro;
        }
    };
    if (has_row) put_row(t, ro_t, rd_t);
    for (int i = t + MG_THREADS; i <= nr + 1; i += MG_THREADS)  // tiles of many short rows
        if (r0 + i <= n) put_row(i, off[r0 + i], doff[r0 + i]);
    if (dlds) {
        if (has_dc) {
            s_dc[t] = dc_raw;
            s_dw[t] = dw_raw;
        }
        for (int q = t + MG_THREADS; q < ndt; q += MG_THREADS) {
            s_dc[q] = dcol[dbase + q];
            s_dw[q] = dw[dbase + q];
        }
    }
    if (wv == 0) {
        // tombstones before e0: counter blocks before its block + a ballot count inside it
        int cd = 0;
#pragma unroll
        for (int q = 0; q < TILE / WAVE; ++q)
            cd += __popcll(ballot(st + q * WAVE + l < e0 && (tbc[q] & DEAD) != 0u));
        if (l == 0) {
            s_base[0] = ro_t;  // off[r0]
            s_base[1] = tb0 + cd;
        }
    }
    __syncthreads();
    int64_t pre = s_base[1];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        int64_t pu = pre;
        for (int q = 0; q < wv; ++q) pu += s_wd[u][q];
        for (int q = 0; q < MG_WAVES; ++q) pre += s_wd[u][q];
        const int j = u * MG_THREADS + t;
        // column of entry j - 1 (lane 0: the last entry of the wave before) and the
        // tombstones before it in its wave (taken while every lane is active)
        const uint32_t pc = (uint32_t)__shfl_up((int32_t)c[u], 1, WAVE);
        const int lp = __popcll(ballot((c[u] & DEAD) != 0u) & lanemask_lt());
        if (j >= ne) continue;
        const int64_t i = e0 + j;
        const int64_t deadG = pu + lp;  // tombstones before entry i
        // row of the entry: last row of the tile that starts at or before j
        int lo = 0, hi = nr;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        const int64_t ro = lo == 0 ? s_base[0] : e0 + s_off[lo];
        const uint32_t cu = c[u];
        const uint32_t cur = cu & ID_MASK;
        const bool dead = cu & DEAD;
        const int dl = s_dlo[lo], dh = s_dlo[lo + 1];  // this row's diff entries (tile-relative)
        // where the entry would land with none of its row's diff entries before it
        const int64_t base0 = i - deadG + dbase + dl;
        if (dl == dh) {
            if (!dead) merge_put(col2, w2, cap, base0, (int32_t)(cu & keep), wt[u], cnt);
            continue;
        }
        // rows with diff entries: interleave them at their insertion points
        auto lower = [&](uint32_t v) -> int {
            return dlds ? lds_lower(s_dc, dl, dh, v) : (int)(lower_sorted(dcol, dbase + dl, dbase + dh, v) - dbase);
        };
        auto put_diff = [&](int q, int64_t o) {
            merge_put(col2, w2, cap, o, (int32_t)((uint32_t)(dlds ? s_dc[q] : dcol[dbase + q]) & keep),
                      dlds ? s_dw[q] : dw[dbase + q], cnt);
        };
        const int bq = lower(cur);
        if (!dead) merge_put(col2, w2, cap, base0 + (bq - dl), (int32_t)(cu & keep), wt[u], cnt);
        int a = dl;
        if (i > ro) {
            const uint32_t p = l > 0 ? pc : (wv > 0 ? s_last[u][wv] : (u > 0 ? s_last[u - 1][MG_WAVES] : s_last[0][0]));
            a = lower((p & ID_MASK) + 1);
        }
        for (int q = a; q < bq; ++q) put_diff(q, base0 + (q - dl));
        const int64_t rend = lo < nr ? e0 + s_off[lo + 1] : s_base[2];
        if (i == rend - 1) {  // after the row's last base entry: the diff tail
            const int64_t after = dead ? 0 : 1;
            for (int q = lower(cur + 1); q < dh; ++q) put_diff(q, base0 + after + (q - dl));
        }
    }
}

// Diff entries of rows whose base part is empty.
__global__ void k_merge_diff_empty(int64_t dm, const uint64_t *dkey, int B, const int64_t *off,
                                   const int64_t *doff, const int32_t *dcol, const int32_t *dw,
                                   const int64_t *off2, int32_t *col2, int32_t *w2, int64_t cap,
                                   uint32_t keep, int64_t *cnt) {
    for (int64_t j = gtid(); j < dm; j += gstride()) {
        int32_t r = (int32_t)(dkey[j] >> B);
        if (off[r] != off[r + 1]) continue;
        int64_t o = off2[r] + (j - doff[r]);
        if (o < 0 || o >= cap) { atomicOr((unsigned long long *)&cnt[C_ERR], 4ull); continue; }
        col2[o] = (int32_t)((uint32_t)dcol[j] & keep);
        w2[o] = dw[j];
    }
}

// Merge direction d into (off2, col2, w2).  side: on the graph's second stream,
// with the merge's own error counter and scan scratch, and without waiting for it
// (merge_side_check reads the counter once the stream is done).  A side merge
// runs beside the post-hooks, which read the unmerged arrays, and its output is
// swapped in after them: it drops the MARK of inserted entries as it copies them,
// which the clearing pass would otherwise do on the merged arrays.  Merges on the
// graph's stream run before the post-hooks and keep MARK (the triangle delta
// weighs inserted arcs by it).
static int merge_into(dg_graph *g, Dir &d, int64_t *off2, int32_t *col2, int32_t *w2, int64_t m2,
                      bool side = false) {
    hipStream_t s = side ? g->aux : g->stream;
    Work &ws = g->ws;
    int64_t *cnt = side ? ws.dcnt_m : ws.dcnt;
    SortWork &sw = side ? ws.sw_m : ws.sw;
    const uint32_t keep = side ? ~MARK : ~0u;
    const int32_t n = g->n;
    const int64_t nblk = ntiles_for(d.m);
    DG_TRY(ws.scan64.ensure((size_t)n + 1 + 2 * (nblk + 2)));
    int64_t *tmpa = ws.scan64.p;
    int64_t *tsin = tmpa + (n + 1);
    int64_t *TB = tsin + (nblk + 2);
    // off2 = exclusive scan of live degrees
    hipLaunchKernelGGL(k_deg_to_i64, dim3(grid_for(n + 1)), dim3(256), 0, s, n, d.deg.p, tmpa);
    DG_TRY(scan_excl_on(s, sw, cnt + C_SORT_ERR, tmpa, off2, n + 1));
    // TB = tombstones before each counter block
    hipLaunchKernelGGL(k_deg_to_i64, dim3(grid_for(nblk + 2)), dim3(256), 0, s, (int32_t)(nblk + 1), d.ttomb.p,
                       tsin);
    DG_TRY(scan_excl_on(s, sw, cnt + C_SORT_ERR, tsin, TB, nblk + 2));
    // merge-path tiles
    const int mt = g->cfg.merge_tile;
    const int items = mt == 512 || mt == 1024 || mt == 2048 ? mt : MG_ITEMS;
    const int64_t nb = ((int64_t)n + d.m + items - 1) / items;
    DG_TRY(ws.mp_row.ensure((size_t)nb + 1));
    DG_TRY(ws.mp_edge.ensure((size_t)nb + 1));
    DG_TRY(ws.mp_doff.ensure(2 * ((size_t)nb + 1)));
    int64_t *mp_dlo = ws.mp_doff.p, *mp_dhi = mp_dlo + (nb + 1);
    hipLaunchKernelGGL(k_mg_partition, dim3(grid_for(nb + 1)), dim3(256), 0, s, d.off.p, d.doff.p, n, d.m, nb,
                       items, ws.mp_row.p, ws.mp_edge.p, mp_dlo, mp_dhi);
    DG_HIP(hipGetLastError());
    DG_TRY(fill_i64(cnt, 0, C_MAXROW, s));  // the longest-row bound stays (rows only shrink here)
    // merge bytes: col+w read 8 per old entry, write 8 per new entry, and per row
    // off and doff (8 each)
    int pm = prof_begin("merge_base", s);
    auto tiles_kernel = items == 512 ? k_merge_tiles<512> : (items == 2048 ? k_merge_tiles<2048> : k_merge_tiles<1024>);
    if (nb > 0)
        hipLaunchKernelGGL(tiles_kernel, dim3((unsigned)nb), dim3(MG_THREADS), 0, s, n, ws.mp_row.p,
                           ws.mp_edge.p, mp_dlo, mp_dhi, d.off.p, d.col.p, d.w.p, d.doff.p, d.dcol.p, d.dw.p, TB, col2, w2,
                           m2, keep, cnt);
    prof_end(pm, s, 8.0 * (double)d.m + 8.0 * (double)m2 + 16.0 * (double)n + 8.0 * (double)d.dm);
    if (d.dm > 0)
        hipLaunchKernelGGL(k_merge_diff_empty, dim3(grid_for(d.dm)), dim3(256), 0, s, d.dm, d.dkey.p,
                           d.keybits, d.off.p, d.doff.p, d.dcol.p, d.dw.p, off2, col2, w2, m2, keep, cnt);
    DG_HIP(hipGetLastError());
    if (side) return DG_OK;
    DG_TRY(counters_read(g));
    if (ws.hcnt[C_ERR]) return set_error(DG_EDEVICE, "merge: inconsistent degree counts (internal error)");
    return DG_OK;
}

// The merge's error counter after a merge on the second stream (waits for it).
static int merge_side_check(dg_graph *g) {
    DG_HIP(hipMemcpyAsync(g->ws.hcnt_m, g->ws.dcnt_m, sizeof(int64_t) * C_COUNT, hipMemcpyDeviceToHost, g->aux));
    DG_HIP(hipStreamSynchronize(g->aux));
    if (g->ws.hcnt_m[C_ERR]) return set_error(DG_EDEVICE, "merge: inconsistent degree counts (internal error)");
    if (g->ws.hcnt_m[C_SORT_ERR]) return set_error(DG_EDEVICE, "merge: scan look-back did not finish (internal error)");
    return DG_OK;
}

// Merged arrays become the base; the diff level and the tombstone counters empty.
static int merge_dir_commit(dg_graph *g, Dir &d, int64_t live) {
    hipStream_t s = g->stream;
    d.off.swap(d.off2);
    d.col.swap(d.col2);
    d.w.swap(d.w2);
    d.m = live;
    d.dm = 0;
    d.tomb_base = 0;
    d.tomb_diff = 0;
    DG_TRY(fill_i64(d.doff.p, 0, g->n + 1, s));
    DG_TRY(fill_i32(d.ntomb.p, 0, g->n + 1, s));
    DG_TRY(d.ttomb.ensure(ntiles_for(live) + 2));
    DG_TRY(fill_i32(d.ttomb.p, 0, ntiles_for(live) + 2, s));
    return DG_OK;
}

static bool merge_needed(const Dir &d) { return d.dm != 0 || d.tomb_base != 0; }

// Merged arrays of direction d into its spare buffers (side: on the second stream).
static int merge_dir_start(dg_graph *g, Dir &d, int64_t live, bool side) {
    DG_TRY(d.off2.ensure(g->n + 1));
    DG_TRY(d.col2.ensure(live + 1));
    DG_TRY(d.w2.ensure(live + 1));
    return merge_into(g, d, d.off2.p, d.col2.p, d.w2.p, live, side);
}

static int merge_dir(dg_graph *g, Dir &d, int64_t live) {
    if (!merge_needed(d)) return DG_OK;
    DG_TRY(merge_dir_start(g, d, live, false));
    return merge_dir_commit(g, d, live);
}

int graph_merge(dg_graph *g) {
    DG_TRY(merge_dir(g, g->fwd, g->m_live));
    if (!g->undirected) DG_TRY(merge_dir(g, g->rev_own, g->m_live));
    DG_HIP(hipStreamSynchronize(g->stream));
    return DG_OK;
}

// ---------------------------------------------------------------- export

__global__ void k_rows_of_entries(int32_t n, int64_t m, const int64_t *off, int32_t *row) {
    for (int64_t i = gtid(); i < m; i += gstride()) row[i] = row_of(off, 0, n - 1, i);
}

int graph_export(dg_graph *g, int64_t *m, int32_t *src, int32_t *dst, int32_t *w) {
    const int64_t arcs = g->m_live;
    const int64_t count = g->undirected ? arcs / 2 : arcs;
    if (!src) {
        *m = count;
        return DG_OK;
    }
    if (*m < count) return set_error(DG_EINVAL, "export capacity %lld < %lld", (long long)*m, (long long)count);
    hipStream_t s = g->stream;
    Dir &d = g->fwd;
    DBuf<int64_t> off2;
    DBuf<int32_t> col2, w2, row;
    DG_TRY(off2.ensure(g->n + 1));
    DG_TRY(col2.ensure(arcs + 1));
    DG_TRY(w2.ensure(arcs + 1));
    DG_TRY(row.ensure(arcs + 1));
    int rc = merge_into(g, d, off2.p, col2.p, w2.p, arcs);
    if (rc == DG_OK && arcs > 0)
        hipLaunchKernelGGL(k_rows_of_entries, dim3(grid_for(arcs)), dim3(256), 0, s, g->n, arcs, off2.p,
                           row.p);
    std::vector<int32_t> hr(arcs), hc(arcs), hw(arcs), hi;
    if (rc == DG_OK && arcs > 0) {
        (void)hipMemcpyAsync(hr.data(), row.p, arcs * 4, hipMemcpyDeviceToHost, s);
        (void)hipMemcpyAsync(hc.data(), col2.p, arcs * 4, hipMemcpyDeviceToHost, s);
        (void)hipMemcpyAsync(hw.data(), w2.p, arcs * 4, hipMemcpyDeviceToHost, s);
        if (g->relabeled) {
            hi.resize(g->n);
            (void)hipMemcpyAsync(hi.data(), g->iperm.p, (size_t)g->n * 4, hipMemcpyDeviceToHost, s);
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    off2.release(); col2.release(); w2.release(); row.release();
    if (rc != DG_OK) return rc;
    if (e != hipSuccess) return set_error(DG_EDEVICE, "export copy failed: %s", hipGetErrorString(e));
    if (!g->relabeled) {
        int64_t o = 0;
        for (int64_t i = 0; i < arcs; ++i) {
            int32_t u = hr[i], v = (int32_t)((uint32_t)hc[i] & ID_MASK);
            if (g->undirected && u > v) continue;
            src[o] = u;
            dst[o] = v;
            if (w) w[o] = hw[i];
            ++o;
        }
        *m = o;
        return DG_OK;
    }
    // caller's ids, sorted again by (src, dst)
    std::vector<std::pair<uint64_t, int32_t>> ed;
    ed.reserve((size_t)count);
    for (int64_t i = 0; i < arcs; ++i) {
        const uint32_t u = (uint32_t)hi[hr[i]], v = (uint32_t)hi[(uint32_t)hc[i] & ID_MASK];
        if (g->undirected && u > v) continue;
        ed.emplace_back(((uint64_t)u << 32) | v, hw[i]);
    }
    std::sort(ed.begin(), ed.end());
    for (size_t o = 0; o < ed.size(); ++o) {
        src[o] = (int32_t)(ed[o].first >> 32);
        dst[o] = (int32_t)(ed[o].first & 0xffffffffu);
        if (w) w[o] = ed[o].second;
    }
    *m = (int64_t)ed.size();
    return DG_OK;
}

// ---------------------------------------------------------------- batch application

// Validation of a whole chunk before any change (rejects self-loops, ids outside
// [0, n), ops other than 0/1 and insert weights outside [1, 2^30)).
__global__ __launch_bounds__(CH_T) void k_validate_batch(int64_t k, const int32_t *s, const int32_t *d,
                                                         const int32_t *w, const uint8_t *op, int32_t n,
                                                         int expect, int64_t *cnt) {
    __shared__ BlockScratch sc;
    int64_t nd = 0, ni = 0;
    bool anybad = false;
    for (int64_t i = gtid(); i < k; i += gstride()) {
        int32_t u = s[i], v = d[i];
        uint8_t o = op[i];
        bool bad = u < 0 || u >= n || v < 0 || v >= n || u == v || o > 1 || (expect >= 0 && o != expect);
        if (o == 1 && w) bad |= (w[i] < 1 || w[i] >= (1 << 30));
        anybad |= bad;
        nd += !bad && o == 0;
        ni += !bad && o == 1;
    }
    if (anybad) atomicOr((unsigned long long *)&cnt[C_ERR], 1ull);
    block_count(&cnt[C_NDEL], nd, sc);
    block_count(&cnt[C_NINS], ni, sc);
}

// Split the chunk into deletion arcs and insertion keys (undirected updates give
// both arcs).  A workgroup takes CH updates, each thread CH_IPT of them strided by
// the workgroup size (coalesced loads); the outputs of one workgroup are one
// contiguous range, in thread order (the order of arcs and keys is free: the keys
// are sorted next, and repeated deletions are told apart by the MARK bit).
__global__ __launch_bounds__(CH_T) void k_expand_batch(int64_t k, const int32_t *s, const int32_t *d,
                                                       const int32_t *w, const uint8_t *op, int B,
                                                       int undirected, const int32_t *perm, int32_t *ddu,
                                                       int32_t *ddv, uint64_t *ikey, int32_t *iw, int64_t *cnt) {
    __shared__ BlockScratch sc;
    const int rep = undirected ? 2 : 1;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < k; c0 += (int64_t)gridDim.x * CH) {
        uint8_t o[CH_IPT];
        int32_t su[CH_IPT], dv[CH_IPT], wt[CH_IPT];
        int64_t nd = 0, ni = 0;
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            const int64_t i = c0 + (int64_t)q * CH_T + threadIdx.x;
            o[q] = i < k ? op[i] : (uint8_t)2;
            su[q] = i < k ? s[i] : 0;
            dv[q] = i < k ? d[i] : 0;
            wt[q] = i < k && w ? w[i] : 1;
            nd += o[q] == 0;
            ni += o[q] == 1;
        }
        int64_t pd = block_reserve(&cnt[C_AUX0], nd * rep, sc);
        int64_t pi = block_reserve(&cnt[C_AUX1], ni * rep, sc);
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            if (o[q] > 1) continue;
            const uint32_t u0 = (uint32_t)(perm ? perm[su[q]] : su[q]), v0 = (uint32_t)(perm ? perm[dv[q]] : dv[q]);
            for (int r = 0; r < rep; ++r) {
                const uint32_t u = r ? v0 : u0, v = r ? u0 : v0;
                if (o[q] == 0) {
                    ddu[pd] = (int32_t)u;
                    ddv[pd] = (int32_t)v;
                    ++pd;
                } else {
                    ikey[pi] = ((uint64_t)u << B) | v;
                    iw[pi] = wt[q];
                    ++pi;
                }
            }
        }
    }
}

// updateCSRDel, first half: find each deletion arc and MARK it (the old graph is
// still intact for the pre-hooks).  The atomic MARK also dedups repeated
// deletions of one arc.  Applied arcs are listed with their slot
// (>= 0: base position, <= -2: diff position -2-p).
__global__ __launch_bounds__(CH_T) void k_mark_deletes(int64_t na, const int32_t *ddu, const int32_t *ddv,
                                                       const int64_t *__restrict__ off, int32_t *col,
                                                       const int64_t *__restrict__ doff, int32_t *dcol,
                                                       int undirected, int32_t *adu, int32_t *adv,
                                                       int64_t *adpos, int32_t *tcu, int32_t *tcv,
                                                       int64_t *cnt) {
    __shared__ BlockScratch sc;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < na; c0 += (int64_t)gridDim.x * CH) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * CH_IPT;
        int32_t u[CH_IPT];
        uint32_t v[CH_IPT];
        bool ok[CH_IPT];
        int64_t p[CH_IPT], r[CH_IPT];
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            ok[q] = i0 + q < na;
            u[q] = ok[q] ? ddu[i0 + q] : 0;
            v[q] = ok[q] ? (uint32_t)ddv[i0 + q] : 0u;
        }
        find_arcs(off, col, doff, dcol, u, v, ok, p, r);  // the diff level only where the base lacks the arc
        int64_t pos[CH_IPT];
        int64_t nap = 0, ntc = 0;
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            pos[q] = -1;  // -1: not applied
            if (i0 + q >= na) continue;
            if (p[q] >= 0) {
                if (!((uint32_t)col[p[q]] & DEAD)) {
                    const uint32_t old = atomicOr((unsigned int *)&col[p[q]], MARK);
                    if (!(old & MARK)) pos[q] = p[q];
                }
            } else if (r[q] >= 0 && !((uint32_t)dcol[r[q]] & DEAD)) {
                const uint32_t old = atomicOr((unsigned int *)&dcol[r[q]], MARK);
                if (!(old & MARK)) pos[q] = -2 - r[q];
            }
            if (pos[q] != -1) {
                ++nap;
                ntc += undirected && (uint32_t)u[q] < v[q];
            }
        }
        int64_t slot = block_reserve(&cnt[C_ADEL], nap, sc);
        int64_t ts = block_reserve(&cnt[C_TCDEL], ntc, sc);
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            if (pos[q] == -1) continue;
            adu[slot] = u[q];
            adv[slot] = (int32_t)v[q];
            adpos[slot] = pos[q];
            ++slot;
            if (undirected && (uint32_t)u[q] < v[q]) {
                tcu[ts] = u[q];
                tcv[ts] = (int32_t)v[q];
                ++ts;
            }
        }
    }
}

// Classify the sorted insertion keys: the first key of each run takes the
// smallest weight of the run; it is IGNORED if the edge is live and not being
// deleted, REVIVED in place if its slot is a tombstone or is being deleted in this
// chunk (delete + insert ends present with the new weight), otherwise NEW.
__global__ __launch_bounds__(CH_T) void k_classify_inserts(int64_t ni, const uint64_t *key, int32_t *iw, int B,
                                   const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                   const int64_t *__restrict__ doff, const int32_t *__restrict__ dcol,
                                   int undirected, int64_t *isnew, int32_t *aiu, int32_t *aiv,
                                   int32_t *aiw, int64_t *aipos, int64_t *cnt) {
    __shared__ BlockScratch sc;
    const uint64_t mask = (1ull << B) - 1;
    int64_t nnew = 0, nign = 0, ndist = 0;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < ni; c0 += (int64_t)gridDim.x * CH) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * CH_IPT;
        int64_t pos[CH_IPT];
        int8_t act[CH_IPT];  // 0 none, 1 new, 2 revive, 3 ignore
        int64_t napp = 0;
        bool head[CH_IPT];
        int32_t u[CH_IPT];
        uint32_t v[CH_IPT];
        int64_t p[CH_IPT], r[CH_IPT];
        // run heads: the smallest weight of the run, then the row bounds
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            const int64_t i = i0 + q;
            head[q] = false;
            u[q] = 0;
            v[q] = 0u;
            if (i >= ni) continue;
            const uint64_t kk = key[i];
            head[q] = i == 0 || kk != key[i - 1];
            if (!head[q]) continue;
            int32_t wt = iw[i];
            for (int64_t j = i + 1; j < ni && key[j] == kk; ++j) wt = min(wt, iw[j]);
            iw[i] = wt;
            u[q] = (int32_t)(kk >> B);
            v[q] = (uint32_t)(kk & mask);
        }
        find_arcs(off, col, doff, dcol, u, v, head, p, r);
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            const int64_t i = i0 + q;
            act[q] = 0;
            pos[q] = -1;
            if (i >= ni) continue;
            if (head[q]) {
                if (p[q] >= 0) {
                    if ((uint32_t)col[p[q]] & (DEAD | MARK)) { act[q] = 2; pos[q] = p[q]; }
                    else act[q] = 3;
                } else if (r[q] >= 0) {
                    if ((uint32_t)dcol[r[q]] & (DEAD | MARK)) { act[q] = 2; pos[q] = -2 - r[q]; }
                    else act[q] = 3;
                } else {
                    act[q] = 1;
                }
                ++ndist;
            }
            isnew[i] = act[q] == 1;
            napp += act[q] == 1 || act[q] == 2;
            nnew += act[q] == 1;
            nign += act[q] != 1 && act[q] != 2;
        }
        int64_t slot = block_reserve(&cnt[C_AINS], napp, sc);
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            if (act[q] != 1 && act[q] != 2) continue;
            const uint64_t kk = key[i0 + q];
            aiu[slot] = (int32_t)(kk >> B);
            aiv[slot] = (int32_t)(kk & mask);
            aiw[slot] = iw[i0 + q];
            aipos[slot] = pos[q];
            ++slot;
        }
    }
    block_count(&cnt[C_NEW], nnew, sc);
    block_count(&cnt[C_IGNINS], nign, sc);
    block_count(&cnt[C_DISTINCT], ndist, sc);
    (void)undirected;
}

__global__ void k_compact_new(int64_t ni, const uint64_t *key, const int32_t *iw, const int64_t *isnew,
                              const int64_t *pos, uint64_t *nkey, int32_t *nw) {
    for (int64_t i = gtid(); i < ni; i += gstride())
        if (isnew[i]) { nkey[pos[i]] = key[i]; nw[pos[i]] = iw[i]; }
}

// TC needs the inserted undirected edges once each.
__global__ __launch_bounds__(CH_T) void k_list_tc_inserts(int64_t na, const int32_t *aiu, const int32_t *aiv,
                                                          int32_t *tcu, int32_t *tcv, int64_t *cnt) {
    __shared__ BlockScratch sc;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < na; c0 += (int64_t)gridDim.x * CH) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * CH_IPT;
        int64_t np = 0;
        for (int q = 0; q < CH_IPT; ++q) np += i0 + q < na && aiu[i0 + q] < aiv[i0 + q];
        int64_t s = block_reserve(&cnt[C_TCINS], np, sc);
        for (int q = 0; q < CH_IPT; ++q) {
            const int64_t i = i0 + q;
            if (i < na && aiu[i] < aiv[i]) {
                tcu[s] = aiu[i];
                tcv[s] = aiv[i];
                ++s;
            }
        }
    }
}

// updateCSRDel, second half: turn the MARKs of applied deletions into tombstones.
__global__ void k_commit_deletes(int64_t na, const int32_t *adu, const int64_t *adpos, int32_t *col,
                                 int32_t *dcol, int32_t *deg, int32_t *ntomb, int32_t *ttomb,
                                 int64_t *cnt) {
    __shared__ BlockScratch sc;
    int64_t nbase = 0, ndiff = 0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool inbase = false, indiff = false;
        if (i < na) {
            int32_t u = adu[i];
            int64_t p = adpos[i];
            if (p >= 0) {
                col[p] = (int32_t)(((uint32_t)col[p] & ~MARK) | DEAD);
                atomicAdd(&ntomb[u], 1);
                atomicAdd(&ttomb[p / TILE], 1);
                inbase = true;
            } else {
                int64_t q = -2 - p;
                dcol[q] = (int32_t)(((uint32_t)dcol[q] & ~MARK) | DEAD);
                indiff = true;
            }
            atomicSub(&deg[u], 1);
        }
        nbase += inbase;
        ndiff += indiff;
    }
    block_count(&cnt[C_AUX2], nbase, sc);
    block_count(&cnt[C_AUX3], ndiff, sc);
}

// Reverse direction of a directed graph: find (v, u) in row v and tombstone it.
__global__ void k_commit_deletes_rev(int64_t na, const int32_t *adu, const int32_t *adv,
                                     const int64_t *__restrict__ off, int32_t *col,
                                     const int64_t *__restrict__ doff, int32_t *dcol, int32_t *deg,
                                     int32_t *ntomb, int32_t *ttomb, int64_t *cnt) {
    __shared__ BlockScratch sc;
    int64_t nbase = 0, ndiff = 0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool inbase = false, indiff = false;
        if (i < na) {
            int32_t u = adu[i], v = adv[i];
            int64_t p = find_sorted(col, off[v], off[v + 1], (uint32_t)u);
            if (p >= 0) {
                col[p] = (int32_t)(((uint32_t)col[p] & ~MARK) | DEAD);
                atomicAdd(&ntomb[v], 1);
                atomicAdd(&ttomb[p / TILE], 1);
                inbase = true;
            } else {
                int64_t q = find_sorted(dcol, doff[v], doff[v + 1], (uint32_t)u);
                if (q >= 0) {
                    dcol[q] = (int32_t)(((uint32_t)dcol[q] & ~MARK) | DEAD);
                    indiff = true;
                }
            }
            if (inbase || indiff) atomicSub(&deg[v], 1);
        }
        nbase += inbase;
        ndiff += indiff;
    }
    block_count(&cnt[C_AUX2], nbase, sc);
    block_count(&cnt[C_AUX3], ndiff, sc);
}

// updateCSRAdd for slots that already exist: revive a tombstone in place
// (sorted hole reuse) with the new weight; NEW arcs only bump the degree here.
// Inserted entries carry MARK until the post-hooks have run.
__global__ __launch_bounds__(CH_T) void k_revive(int64_t na, const int32_t *aiu, const int32_t *aiv,
                                                 const int32_t *aiw, const int64_t *aipos, int reverse,
                                                 const int64_t *__restrict__ off, int32_t *col, int32_t *w,
                                                 const int64_t *__restrict__ doff, int32_t *dcol, int32_t *dw,
                                                 int32_t *deg, int32_t *ntomb, int32_t *ttomb, int B,
                                                 uint64_t *rkey, int32_t *rw, int64_t *cnt) {
    __shared__ BlockScratch sc;
    int64_t nrev = 0;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < na; c0 += (int64_t)gridDim.x * CH) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * CH_IPT;
        int32_t r[CH_IPT];
        uint32_t c[CH_IPT];
        int64_t p[CH_IPT];
        int64_t nnew = 0;
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            const bool ok = i0 + q < na;
            const int32_t u = ok ? aiu[i0 + q] : 0, v = ok ? aiv[i0 + q] : 0;
            r[q] = reverse ? v : u;
            c[q] = (uint32_t)(reverse ? u : v);
            p[q] = ok ? aipos[i0 + q] : -1;
            nnew += ok && p[q] == -1;
        }
        if (reverse) {  // locate the revived slots in the reverse store
            int64_t pb[CH_IPT], pd[CH_IPT];
            bool look[CH_IPT];
#pragma unroll
            for (int q = 0; q < CH_IPT; ++q) look[q] = p[q] != -1;
            find_arcs(off, col, doff, dcol, r, c, look, pb, pd);
            // A tombstone revived in the forward store may have no counterpart in the
            // reverse store: each direction reuses its vacant slots on its own, so the
            // reverse tombstone of this arc may hold another arc by now.  Such an arc
            // is new to the reverse store (-1: it joins the reverse NEW keys).
#pragma unroll
            for (int q = 0; q < CH_IPT; ++q)
                if (p[q] != -1) p[q] = pb[q] >= 0 ? pb[q] : (pd[q] >= 0 ? -2 - pd[q] : -1);
            nnew = 0;
#pragma unroll
            for (int q = 0; q < CH_IPT; ++q) nnew += i0 + q < na && p[q] == -1;
        }
        // degree bumps are summed over runs of one row within the thread's elements
        int32_t run_r = -1, run_n = 0;
#pragma unroll
        for (int q = 0; q < CH_IPT; ++q) {
            if (i0 + q >= na) continue;
            const int32_t wt = aiw[i0 + q];
            if (p[q] >= 0) {
                col[p[q]] = (int32_t)(c[q] | MARK);
                w[p[q]] = wt;
                atomicSub(&ntomb[r[q]], 1);
                atomicSub(&ttomb[p[q] / TILE], 1);
                ++nrev;
            } else if (p[q] <= -2) {
                const int64_t d = -2 - p[q];
                dcol[d] = (int32_t)(c[q] | MARK);
                dw[d] = wt;
            }
            if (r[q] != run_r) {
                if (run_n) atomicAdd(&deg[run_r], run_n);
                run_r = r[q];
                run_n = 0;
            }
            ++run_n;
        }
        if (run_n) atomicAdd(&deg[run_r], run_n);
        if (rkey) {
            // NEW arcs of this thread's elements, in element order, for the reverse diff
            int64_t s = block_reserve(&cnt[C_AUX1], nnew, sc);
#pragma unroll
            for (int q = 0; q < CH_IPT; ++q) {
                if (i0 + q < na && p[q] == -1) {
                    rkey[s] = ((uint64_t)(uint32_t)r[q] << B) | c[q];
                    rw[s] = aiw[i0 + q];
                    ++s;
                }
            }
        }
    }
    block_count(&cnt[C_AUX2], nrev, sc);
}

// Sorted hole reuse (Section "Modified Graph Representation: diff-CSR": a new edge
// takes a vacant, tombstoned slot of its row when one is available, and goes to
// the diff-CSR otherwise).  Rows stay sorted by neighbour id, tombstones included,
// so a NEW key v of row u may take a tombstone only next to its sorted position:
// the slot just before it (the largest id below v) or just after it (the smallest
// id above v).  NEW keys are sorted and distinct, and the slot a key wants never
// decreases along a row, so the keys wanting one slot are consecutive and the
// first of them takes it.  Runs after the revivals (a revived slot is live again
// and no longer wanted) and reads only: the writes follow in k_vacancy_fill.
__device__ __forceinline__ int64_t vacancy_of(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                              int32_t u, uint32_t v) {
    const int64_t lo = off[u], hi = off[u + 1];
    if (lo == hi) return -1;
    const int64_t p = lower_sorted(col, lo, hi, v);
    // the key's own tombstone first (a reverse-store arc whose forward tombstone was
    // revived while this one was not taken): reviving it keeps ids distinct
    if (p < hi && ((uint32_t)col[p] & (DEAD | ID_MASK)) == (DEAD | v)) return p;
    if (p > lo && ((uint32_t)col[p - 1] & DEAD)) return p - 1;
    if (p < hi && ((uint32_t)col[p] & DEAD)) return p;
    return -1;
}

// slot[j] = the base slot NEW key j takes, or -1 (it goes to the diff level);
// todiff[j] = 1 for the latter (the compaction's flags, with todiff[nk] = 0).
__global__ void k_vacancy_claim(int64_t nk, const uint64_t *nkey, int B, const int64_t *__restrict__ off,
                                const int32_t *__restrict__ col, int64_t *slot, int64_t *todiff) {
    const uint64_t mask = (1ull << B) - 1;
    for (int64_t j = gtid(); j <= nk; j += gstride()) {
        if (j == nk) {
            todiff[j] = 0;
            continue;
        }
        const uint64_t k = nkey[j];
        const int32_t u = (int32_t)(k >> B);
        int64_t c = vacancy_of(off, col, u, (uint32_t)(k & mask));
        if (c >= 0 && j > 0 && (int32_t)(nkey[j - 1] >> B) == u &&
            vacancy_of(off, col, u, (uint32_t)(nkey[j - 1] & mask)) == c)
            c = -1;  // an earlier key of the row takes this slot
        slot[j] = c;
        todiff[j] = c < 0;
    }
}

// Write the taken slots (MARKed like every fresh insert until the post-hooks end).
__global__ void k_vacancy_fill(int64_t nk, const uint64_t *nkey, const int32_t *nw, int B, const int64_t *slot,
                               int32_t *col, int32_t *w, int32_t *ntomb, int32_t *ttomb, int64_t *cnt) {
    __shared__ BlockScratch sc;
    const uint64_t mask = (1ull << B) - 1;
    int64_t filled = 0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nk; base += gstride()) {
        const int64_t j = base + threadIdx.x;
        if (j < nk && slot[j] >= 0) {
            const int64_t c = slot[j];
            col[c] = (int32_t)((uint32_t)(nkey[j] & mask) | MARK);
            w[c] = nw[j];
            atomicSub(&ntomb[(int32_t)(nkey[j] >> B)], 1);
            atomicSub(&ttomb[c / TILE], 1);
            ++filled;
        }
    }
    block_count(&cnt[C_AUX1], filled, sc);
}

__global__ void k_vacancy_rest(int64_t nk, const uint64_t *nkey, const int32_t *nw, const int64_t *todiff,
                               const int64_t *pos, uint64_t *okey, int32_t *ow) {
    for (int64_t j = gtid(); j < nk; j += gstride())
        if (todiff[j]) {
            okey[pos[j]] = nkey[j];
            ow[pos[j]] = nw[j];
        }
}

// Drop MARK from the entries this chunk inserted.
__global__ void k_clear_marks(int64_t na, const int32_t *aiu, const int32_t *aiv, int reverse,
                              const int64_t *__restrict__ off, int32_t *col,
                              const int64_t *__restrict__ doff, int32_t *dcol) {
    for (int64_t i = gtid(); i < na; i += gstride()) {
        int32_t r = reverse ? aiv[i] : aiu[i];
        int32_t c = reverse ? aiu[i] : aiv[i];
        int64_t p = find_sorted(col, off[r], off[r + 1], (uint32_t)c);
        if (p >= 0) {
            col[p] = (int32_t)((uint32_t)col[p] & ~MARK);
        } else {
            int64_t q = find_sorted(dcol, doff[r], doff[r + 1], (uint32_t)c);
            if (q >= 0) dcol[q] = (int32_t)((uint32_t)dcol[q] & ~MARK);
        }
    }
}

// Diff rebuild: merge the live old diff entries with the sorted NEW keys (keys
// are distinct, so each side's output slot is its rank plus the count of smaller
// keys on the other side) and drop the tombstoned diff entries.
__global__ void k_live_flags(int64_t dm, const int32_t *dcol, int64_t *flags) {
    for (int64_t i = gtid(); i <= dm; i += gstride())
        flags[i] = i < dm ? !((uint32_t)dcol[i] & DEAD) : 0;
}

__global__ void k_diff_old(int64_t dm, const uint64_t *dkey, const int32_t *dcol, const int32_t *dw,
                           const int64_t *rank, const uint64_t *nkey, int64_t nk, uint64_t *dkey2,
                           int32_t *dcol2, int32_t *dw2, int64_t cap) {
    for (int64_t i = gtid(); i < dm; i += gstride()) {
        if ((uint32_t)dcol[i] & DEAD) continue;
        int64_t p = rank[i] + lower_key(nkey, 0, nk, dkey[i]);
        if (p >= cap) continue;
        dkey2[p] = dkey[i];
        dcol2[p] = dcol[i];
        dw2[p] = dw[i];
    }
}

__global__ void k_diff_new(int64_t nk, const uint64_t *nkey, const int32_t *nw, const uint64_t *dkey,
                           int64_t dm, const int64_t *rank, int B, uint64_t *dkey2, int32_t *dcol2,
                           int32_t *dw2, int64_t cap) {
    const uint64_t mask = (1ull << B) - 1;
    for (int64_t j = gtid(); j < nk; j += gstride()) {
        int64_t p = j + rank[lower_key(dkey, 0, dm, nkey[j])];
        if (p >= cap) continue;
        dkey2[p] = nkey[j];
        dcol2[p] = (int32_t)((uint32_t)(nkey[j] & mask) | MARK);
        dw2[p] = nw[j];
    }
}

static int diff_rebuild(dg_graph *g, Dir &d, const uint64_t *nkey, const int32_t *nw, int64_t nk,
                        int64_t killed) {
    if (nk == 0 && killed == 0) return DG_OK;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int64_t dm = d.dm;
    // the diff level grows batch by batch until a merge: grow its scratch and spares
    // by doubling, so that a device reallocation (whose free synchronises the
    // device) is rare
    if (2 * ((size_t)dm + 1) > ws.scan64.cap)
        DG_TRY(ws.scan64.ensure(std::max(2 * ((size_t)dm + 1), 2 * ws.scan64.cap)));
    int64_t *flags = ws.scan64.p;
    int64_t *rank = flags + (dm + 1);
    hipLaunchKernelGGL(k_live_flags, dim3(grid_for(dm + 1)), dim3(256), 0, s, dm, d.dcol.p, flags);
    DG_TRY(scan_excl(g, flags, rank, dm + 1));
    const int64_t live = dm - killed;
    const int64_t dm2 = live + nk;
    if ((size_t)dm2 + 1 > d.dkey2.cap) {
        // Both generations of the level (it alternates with its spare every batch)
        // are sized at their first growth for a full level at the merge threshold,
        // plus two batches: otherwise a level that grows by one batch's new keys
        // each time reallocates almost every batch, and each free synchronises
        // the device.  (A threshold outside (0, 1) falls back to doubling.)
        size_t want = std::max((size_t)dm2 + 1, 2 * d.dkey2.cap);
        const double thr = g->cfg.merge_threshold;
        if (thr > 0.0 && thr < 1.0)
            want = std::max(want, (size_t)(thr * (double)std::max<int64_t>(g->m_live, 1)) + 2 * (size_t)nk + 1);
        DG_TRY(d.dkey2.ensure(want));
        DG_TRY(d.dcol2.ensure(want));
        DG_TRY(d.dw2.ensure(want));
    }
    DG_TRY(d.dcol2.ensure(dm2 + 1));
    DG_TRY(d.dw2.ensure(dm2 + 1));
    if (dm > 0)
        hipLaunchKernelGGL(k_diff_old, dim3(grid_for(dm)), dim3(256), 0, s, dm, d.dkey.p, d.dcol.p,
                           d.dw.p, rank, nkey, nk, d.dkey2.p, d.dcol2.p, d.dw2.p, dm2);
    if (nk > 0)
        hipLaunchKernelGGL(k_diff_new, dim3(grid_for(nk)), dim3(256), 0, s, nk, nkey, nw, d.dkey.p, dm,
                           rank, d.keybits, d.dkey2.p, d.dcol2.p, d.dw2.p, dm2);
    hipLaunchKernelGGL(k_row_offsets, dim3(grid_for(g->n + 1)), dim3(256), 0, s, g->n, d.dkey2.p, dm2,
                       d.keybits, d.doff.p);
    if (nk > 0)
        hipLaunchKernelGGL(k_diff_row_max, dim3(grid_for(nk)), dim3(256), 0, s, nk, nkey, d.keybits, d.off.p,
                           d.doff.p, g->ws.dcnt + C_MAXROW);
    DG_HIP(hipGetLastError());
    d.dkey.swap(d.dkey2);
    d.dcol.swap(d.dcol2);
    d.dw.swap(d.dw2);
    d.dm = dm2;
    d.tomb_diff = 0;
    return DG_OK;
}

// Hole reuse for one direction: NEW keys (sorted, distinct) take the tombstoned
// slots next to their sorted positions where they can; *out / *out_w / *out_n are
// the keys left for the diff level.
static int fill_vacancies(dg_graph *g, Dir &d, const uint64_t *nkey, const int32_t *nw, int64_t nk,
                          const uint64_t **out, const int32_t **out_w, int64_t *out_n) {
    *out = nkey;
    *out_w = nw;
    *out_n = nk;
    if (nk <= 0 || d.tomb_base <= 0 || g->cfg.diff_only) return DG_OK;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    DG_TRY(ws.vslot.ensure(2 * ((size_t)nk + 1)));
    DG_TRY(ws.vkey.ensure((size_t)nk + 1));
    DG_TRY(ws.vw.ensure((size_t)nk + 1));
    int64_t *slot = ws.vslot.p, *todiff = ws.vslot.p + (nk + 1);
    DG_TRY(ws.vpos.ensure((size_t)nk + 1));
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_vacancy_claim, dim3(grid_for(nk + 1)), dim3(256), 0, s, nk, nkey, d.keybits, d.off.p,
                       d.col.p, slot, todiff);
    hipLaunchKernelGGL(k_vacancy_fill, dim3(grid_for(nk)), dim3(256), 0, s, nk, nkey, nw, d.keybits, slot,
                       d.col.p, d.w.p, d.ntomb.p, d.ttomb.p, ws.dcnt);
    DG_HIP(hipGetLastError());
    DG_TRY(scan_excl(g, todiff, ws.vpos.p, nk + 1));
    hipLaunchKernelGGL(k_vacancy_rest, dim3(grid_for(nk)), dim3(256), 0, s, nk, nkey, nw, todiff, ws.vpos.p,
                       ws.vkey.p, ws.vw.p);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    const int64_t filled = g->ws.hcnt[C_AUX1];
    d.tomb_base -= filled;
    *out = ws.vkey.p;
    *out_w = ws.vw.p;
    *out_n = nk - filled;
    return DG_OK;
}

// Wrappers that time a phase with HIP events on the graph's stream.
struct PhaseTimer {
    dg_graph *g;
    int a, b;
    float *acc;
    PhaseTimer(dg_graph *g_, int slot, float *acc_) : g(g_), a(2 * slot), b(2 * slot + 1), acc(acc_) {
        (void)hipEventRecord(g->ws.ev[a], g->stream);
    }
    void stop() {
        (void)hipEventRecord(g->ws.ev[b], g->stream);
        (void)hipEventSynchronize(g->ws.ev[b]);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, g->ws.ev[a], g->ws.ev[b]);
        if (acc) *acc += ms;
    }
};

int apply_chunk(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst, const int32_t *w,
                const uint8_t *op, bool dev, dg_batch_stats *st, int expect_op) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    Dir &F = g->fwd;
    Dir &R = *g->rev;
    const bool und = g->undirected;
    const int B = F.keybits;
    dg_batch_stats dummy{};
    if (!st) st = &dummy;
    PhaseTimer t_all(g, 7, &st->t_total_ms);
    PhaseTimer t_val(g, 0, &st->t_validate_ms);

    // ---- stage the chunk on the device
    const int32_t *ds = src, *dd = dst, *dw = w;
    const uint8_t *dop = op;
    if (!dev) {
        DG_TRY(ws.bsrc.ensure(k + 1));
        DG_TRY(ws.bdst.ensure(k + 1));
        DG_TRY(ws.bop.ensure(k + 1));
        DG_HIP(hipMemcpyAsync(ws.bsrc.p, src, k * 4, hipMemcpyHostToDevice, s));
        DG_HIP(hipMemcpyAsync(ws.bdst.p, dst, k * 4, hipMemcpyHostToDevice, s));
        DG_HIP(hipMemcpyAsync(ws.bop.p, op, k, hipMemcpyHostToDevice, s));
        ds = ws.bsrc.p;
        dd = ws.bdst.p;
        dop = ws.bop.p;
        if (w) {
            DG_TRY(ws.bw.ensure(k + 1));
            DG_HIP(hipMemcpyAsync(ws.bw.p, w, k * 4, hipMemcpyHostToDevice, s));
            dw = ws.bw.p;
        }
    }
    // ---- validate and count (no change to the graph before this passes)
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_validate_batch, dim3(grid_for(k)), dim3(256), 0, s, k, ds, dd, dw, dop, g->n,
                       expect_op, ws.dcnt);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    if (ws.hcnt[C_ERR]) {
        t_val.stop();
        t_all.stop();
        return set_error(DG_EINVAL, "batch holds a self-loop, an id outside [0,n), an op other than 0/1 (or "
                                    "other than the partially dynamic mode's) or a weight outside [1,2^30)");
    }
    const int rep = und ? 2 : 1;
    const int64_t nda = ws.hcnt[C_NDEL] * rep, nia = ws.hcnt[C_NINS] * rep;
    DG_TRY(ws.ddu.ensure(nda + 1)); DG_TRY(ws.ddv.ensure(nda + 1));
    DG_TRY(ws.adu.ensure(nda + 1)); DG_TRY(ws.adv.ensure(nda + 1)); DG_TRY(ws.adpos.ensure(nda + 1));
    DG_TRY(ws.ikey.ensure(nia + 1)); DG_TRY(ws.ikey_s.ensure(nia + 1));
    DG_TRY(ws.iw.ensure(nia + 1)); DG_TRY(ws.iw_s.ensure(nia + 1));
    DG_TRY(ws.aiu.ensure(nia + 1)); DG_TRY(ws.aiv.ensure(nia + 1)); DG_TRY(ws.aiw.ensure(nia + 1));
    DG_TRY(ws.aipos.ensure(nia + 1));
    DG_TRY(ws.nkey.ensure(nia + 1)); DG_TRY(ws.nw.ensure(nia + 1));
    DG_TRY(ws.rkey.ensure(nia + 1)); DG_TRY(ws.rkey_s.ensure(nia + 1));
    DG_TRY(ws.rw.ensure(nia + 1)); DG_TRY(ws.rw_s.ensure(nia + 1));
    DG_TRY(ws.tcu.ensure(nda + nia + 1)); DG_TRY(ws.tcv.ensure(nda + nia + 1));
    DG_TRY(ws.scan64.ensure(2 * ((size_t)nia + 1)));
    const int32_t *perm = g->relabeled ? g->perm.p : nullptr;  // caller's ids to internal ids
    hipLaunchKernelGGL(k_expand_batch, dim3(grid_ch(k)), dim3(256), 0, s, k, ds, dd, dw, dop, B, (int)und, perm,
                       ws.ddu.p, ws.ddv.p, ws.ikey.p, ws.iw.p, ws.dcnt);
    DG_HIP(hipGetLastError());
    DG_TRY(sort_pairs(g, ws.ikey.p, ws.ikey_s.p, ws.iw.p, ws.iw_s.p, nia, 2 * B));
    // ---- updateCSRDel (mark) and insert classification against the old graph
    if (nda > 0)
        hipLaunchKernelGGL(k_mark_deletes, dim3(grid_ch(nda)), dim3(256), 0, s, nda, ws.ddu.p, ws.ddv.p,
                           F.off.p, F.col.p, F.doff.p, F.dcol.p, (int)und, ws.adu.p, ws.adv.p, ws.adpos.p,
                           ws.tcu.p, ws.tcv.p, ws.dcnt);
    int64_t *isnew = ws.scan64.p, *newpos = ws.scan64.p + (nia + 1);
    if (nia > 0)
        hipLaunchKernelGGL(k_classify_inserts, dim3(grid_ch(nia)), dim3(256), 0, s, nia, ws.ikey_s.p,
                           ws.iw_s.p, B, F.off.p, F.col.p, F.doff.p, F.dcol.p, (int)und, isnew, ws.aiu.p,
                           ws.aiv.p, ws.aiw.p, ws.aipos.p, ws.dcnt);
    DG_HIP(hipGetLastError());
    if (nia > 0) {
        DG_TRY(scan_excl(g, isnew, newpos, nia));
        hipLaunchKernelGGL(k_compact_new, dim3(grid_for(nia)), dim3(256), 0, s, nia, ws.ikey_s.p,
                           ws.iw_s.p, isnew, newpos, ws.nkey.p, ws.nw.p);
        DG_HIP(hipGetLastError());
    }
    DG_TRY(counters_read(g));
    const int64_t adel = ws.hcnt[C_ADEL], ains = ws.hcnt[C_AINS], nnew = ws.hcnt[C_NEW];
    const int64_t tcdel = ws.hcnt[C_TCDEL];
    t_val.stop();

    // ---- pre-hooks on the old graph (deleted arcs still present, MARKed)
    for (dg_query *q : g->queries) {
        if (q->kind == Q_SSSP) {
            PhaseTimer t(g, 2, &st->t_sssp_ms);
            DG_TRY(sssp_pre_delete(q, adel));
            t.stop();
        } else if (q->kind == Q_TC && tcdel > 0) {
            PhaseTimer t(g, 4, &st->t_tc_ms);
            uint64_t sum6 = 0;
            int64_t walked = 0;
            DG_TRY(tc_delta(g, ws.tcu.p, ws.tcv.p, tcdel, &sum6, &walked));
            st->edges_traversed += walked;
            q->tc -= sum6 / 6;
            st->tc_removed += (int64_t)(sum6 / 6);
            t.stop();
        }
    }

    // ---- commit deletions, revive slots, rebuild the diff (both directions)
    // The commits count into slots of their own (KILL_F, KILL_R: C_AUX2 and C_AUX3
    // relative to them), so one read after the revivals serves both passes.
    PhaseTimer t_upd(g, 1, &st->t_update_ms);
    constexpr int KILL_F = 16, KILL_R = 18;  // counts at 32..35, clear of every other use
    static_assert(C_AUX3 + KILL_R < C_SORT_ERR && C_AUX2 + KILL_F > C_EDGES, "kill counts have free slots");
    DG_TRY(counters_clear(g));
    if (adel > 0) {
        hipLaunchKernelGGL(k_commit_deletes, dim3(grid_for(adel)), dim3(256), 0, s, adel, ws.adu.p,
                           ws.adpos.p, F.col.p, F.dcol.p, F.deg.p, F.ntomb.p, F.ttomb.p, ws.dcnt + KILL_F);
        if (!und)
            hipLaunchKernelGGL(k_commit_deletes_rev, dim3(grid_for(adel)), dim3(256), 0, s, adel, ws.adu.p,
                               ws.adv.p, R.off.p, R.col.p, R.doff.p, R.dcol.p, R.deg.p, R.ntomb.p,
                               R.ttomb.p, ws.dcnt + KILL_R);
    }
    if (ains > 0) {
        hipLaunchKernelGGL(k_revive, dim3(grid_ch(ains)), dim3(256), 0, s, ains, ws.aiu.p, ws.aiv.p,
                           ws.aiw.p, ws.aipos.p, 0, F.off.p, F.col.p, F.w.p, F.doff.p, F.dcol.p, F.dw.p,
                           F.deg.p, F.ntomb.p, F.ttomb.p, B, (uint64_t *)nullptr, (int32_t *)nullptr,
                           ws.dcnt);
        if (!und)
            hipLaunchKernelGGL(k_revive, dim3(grid_ch(ains)), dim3(256), 0, s, ains, ws.aiu.p, ws.aiv.p,
                               ws.aiw.p, ws.aipos.p, 1, R.off.p, R.col.p, R.w.p, R.doff.p, R.dcol.p,
                               R.dw.p, R.deg.p, R.ntomb.p, R.ttomb.p, B, ws.rkey.p, ws.rw.p,
                               ws.dcnt + 8);
        if (und)
            hipLaunchKernelGGL(k_list_tc_inserts, dim3(grid_ch(ains)), dim3(256), 0, s, ains, ws.aiu.p,
                               ws.aiv.p, ws.tcu.p + tcdel, ws.tcv.p + tcdel, ws.dcnt);
    }
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    const int64_t killed_base_f = ws.hcnt[C_AUX2 + KILL_F], killed_diff_f = ws.hcnt[C_AUX3 + KILL_F];
    const int64_t killed_base_r = und ? 0 : ws.hcnt[C_AUX2 + KILL_R];
    const int64_t killed_diff_r = und ? 0 : ws.hcnt[C_AUX3 + KILL_R];
    const int64_t revived_base_f = ws.hcnt[C_AUX2];
    const int64_t revived_base_r = und ? 0 : ws.hcnt[C_AUX2 + 8];
    // arcs new to the reverse store: the forward NEW arcs plus revivals whose reverse
    // tombstone another arc has taken since
    const int64_t nnew_r = und ? 0 : ws.hcnt[C_AUX1 + 8];
    const int64_t tcins = ws.hcnt[C_TCINS];
    F.tomb_base += killed_base_f - revived_base_f;
    {
        const uint64_t *fk;
        const int32_t *fw;
        int64_t fn;
        DG_TRY(fill_vacancies(g, F, ws.nkey.p, ws.nw.p, nnew, &fk, &fw, &fn));
        DG_TRY(diff_rebuild(g, F, fk, fw, fn, killed_diff_f));
    }
    if (!und) {
        R.tomb_base += killed_base_r - revived_base_r;
        DG_TRY(sort_pairs(g, ws.rkey.p, ws.rkey_s.p, ws.rw.p, ws.rw_s.p, nnew_r, 2 * B));
        const uint64_t *rk;
        const int32_t *rw;
        int64_t rn;
        DG_TRY(fill_vacancies(g, R, ws.rkey_s.p, ws.rw_s.p, nnew_r, &rk, &rw, &rn));
        DG_TRY(diff_rebuild(g, R, rk, rw, rn, killed_diff_r));
    }
    g->m_live += ains - adel;
    t_upd.stop();

    // ---- merge policy (Section 3.5)
    // With only SSSP queries attached, a merge runs beside their updates.
    bool side_merge = !g->queries.empty(), merge_pending = false, merge_f = false, merge_r = false;
    for (dg_query *q : g->queries) side_merge &= q->kind == Q_SSSP;
    {
        double thr = g->cfg.merge_threshold;
        double live = (double)(g->m_live > 0 ? g->m_live : 1);
        bool need = thr < 0 ? (F.dm + F.tomb_base > 0)
                            : ((double)(F.dm + F.tomb_base) > thr * live ||
                               (!und && (double)(R.dm + R.tomb_base) > thr * live));
        // merge period: also merge after cfg.merge_period batches since the last one
        g->since_merge += 1;
        if (g->cfg.merge_period > 0 && g->since_merge >= g->cfg.merge_period &&
            (F.dm + F.tomb_base > 0 || (!und && R.dm + R.tomb_base > 0)))
            need = true;
        if (need) {
            g->since_merge = 0;
            if (side_merge) {
                // the merge writes the spare arrays on the second stream while the
                // SSSP updates read the unmerged ones; the swap waits for both
                if (!g->aux) {
                    DG_HIP(hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking));
                    DG_HIP(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
                    DG_HIP(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
                }
                merge_f = merge_needed(F);
                merge_r = !und && merge_needed(g->rev_own);
                DG_HIP(hipEventRecord(g->ev_fork, s));
                DG_HIP(hipStreamWaitEvent(g->aux, g->ev_fork, 0));
                DG_HIP(hipEventRecord(ws.ev[6], g->aux));
                if (merge_f) DG_TRY(merge_dir_start(g, F, g->m_live, true));
                if (merge_r) DG_TRY(merge_dir_start(g, g->rev_own, g->m_live, true));
                DG_HIP(hipEventRecord(ws.ev[7], g->aux));
                merge_pending = true;
            } else {
                PhaseTimer t(g, 3, &st->t_merge_ms);
                DG_TRY(merge_dir(g, F, g->m_live));
                if (!und) DG_TRY(merge_dir(g, g->rev_own, g->m_live));
                t.stop();
            }
            st->merged += 1;
        }
    }

    // ---- post-hooks on the new graph
    // With PageRank and frontier-step SSSP queries both attached, the SSSP updates
    // run on a second stream while the PageRank steps stream on this one: the
    // SSSP rounds are latency-bound and leave the device mostly idle.
    dg_query *prq = nullptr;
    bool has_sssp = false;
    for (dg_query *q : g->queries) {
        if (q->kind == Q_PR && !prq) prq = q;
        has_sssp |= q->kind == Q_SSSP;
    }
    if (prq && has_sssp && g->cfg.sssp_persistent != 1) {
        if (!g->aux) {
            DG_HIP(hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking));
            DG_HIP(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
            DG_HIP(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
        }
        DG_HIP(hipEventRecord(g->ev_fork, s));  // the updated graph
        SideWork side;
        side.fn = [&]() -> int {
            // beside the steps: wait for the update only; after them: for everything so far
            if (!side.beside) DG_HIP(hipEventRecord(g->ev_fork, s));
            DG_HIP(hipStreamWaitEvent(g->aux, g->ev_fork, 0));
            g->stream = g->aux;
            int rc = DG_OK;
            for (dg_query *q : g->queries) {
                if (q->kind != Q_SSSP) continue;
                PhaseTimer t(g, 2, &st->t_sssp_ms);
                rc = sssp_post_update(q, adel, ains, st);
                t.stop();
                if (rc != DG_OK) break;
            }
            (void)hipEventRecord(g->ev_join, g->aux);
            (void)wait_stream(g, g->aux);
            g->stream = s;
            if (rc == DG_OK) DG_HIP(hipStreamWaitEvent(s, g->ev_join, 0));
            return rc;
        };
        PhaseTimer t(g, 5, &st->t_pr_ms);
        DG_TRY(pr_post_update(prq, adel, ains, st, &side));
        t.stop();
    }
    for (dg_query *q : g->queries) {
        if (prq && has_sssp && g->cfg.sssp_persistent != 1 && (q == prq || q->kind == Q_SSSP)) continue;
        if (q->kind == Q_SSSP) {
            PhaseTimer t(g, 2, &st->t_sssp_ms);
            DG_TRY(sssp_post_update(q, adel, ains, st));
            t.stop();
        } else if (q->kind == Q_PR) {
            PhaseTimer t(g, 5, &st->t_pr_ms);
            DG_TRY(pr_post_update(q, adel, ains, st));
            t.stop();
        } else if (q->kind == Q_TC && tcins > 0) {
            PhaseTimer t(g, 4, &st->t_tc_ms);
            uint64_t sum6 = 0;
            int64_t walked = 0;
            DG_TRY(tc_delta(g, ws.tcu.p + tcdel, ws.tcv.p + tcdel, tcins, &sum6, &walked));
            st->edges_traversed += walked;
            q->tc += sum6 / 6;
            st->tc_added += (int64_t)(sum6 / 6);
            t.stop();
        }
    }
    // ---- a merge beside the SSSP updates: check it, then swap in the merged arrays
    if (merge_pending) {
        DG_TRY(merge_side_check(g));
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ws.ev[6], ws.ev[7]) == hipSuccess) st->t_merge_ms += ms;
        if (merge_f) DG_TRY(merge_dir_commit(g, F, g->m_live));
        if (merge_r) DG_TRY(merge_dir_commit(g, g->rev_own, g->m_live));
    }
    // ---- drop the MARKs of inserted entries (a side merge dropped them in the
    // arrays it replaced)
    if (ains > 0) {
        if (!merge_f)
            hipLaunchKernelGGL(k_clear_marks, dim3(grid_for(ains)), dim3(256), 0, s, ains, ws.aiu.p, ws.aiv.p,
                               0, F.off.p, F.col.p, F.doff.p, F.dcol.p);
        if (!und && !merge_r)
            hipLaunchKernelGGL(k_clear_marks, dim3(grid_for(ains)), dim3(256), 0, s, ains, ws.aiu.p,
                               ws.aiv.p, 1, R.off.p, R.col.p, R.doff.p, R.dcol.p);
        DG_HIP(hipGetLastError());
    }
    t_all.stop();
    const int64_t div = und ? 2 : 1;
    st->updates += k;
    st->deleted += adel / div;
    st->inserted += ains / div;
    st->ignored_del += (nda - adel) / div;
    st->ignored_ins += (nia - ains) / div;
    st->diff_entries = F.dm;
    st->tombstones = F.tomb_base;
    st->chunks += 1;
    return DG_OK;
}

}  // namespace dg
