// Triangle counting: static count and the delta for a batch (undirected graphs).
//
// Delta (Appendix A, DynTC: Decremental runs on the old graph, Incremental on the
// new one).  For a changed edge {a, b} every common neighbour c closes a
// triangle {a, b, c}; if k of that triangle's three edges are in the batch, the
// triangle is met once from each of them, so each meeting adds 6 / k and the sum
// over all changed edges is 6x the number of changed triangles -- the listing's
// count1/2 + count2/4 + count3/6 with every edge taken once instead of twice.
// An edge is "in the batch" when its entry carries MARK: deletions carry it
// between marking and commit (so the old graph still holds them), insertions
// from insertion until the post-hooks are done -- the edge flags modified_del /
// modified_add of the listing.
//
// Static (comparator; Appendix A staticTC counts every triangle once by vertex
// order): here vertices are ranked by (degree, id), every edge is oriented from
// its lower- to its higher-ranked end, and a triangle is counted once at its
// lowest-ranked vertex by intersecting two forward lists -- the standard forward
// algorithm, whose degree ordering bounds every forward list by sqrt(2m) on skewed
// graphs.
#include <algorithm>

#include "dg_device.h"

namespace dg {

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

struct RowRef {
    int64_t ob, db, od, dd;  // base start/len, diff start/len
};

__device__ __forceinline__ RowRef row_ref(const int64_t *off, const int64_t *doff, int32_t v) {
    RowRef r;
    r.ob = off[v];
    r.db = off[v + 1] - r.ob;
    r.od = doff[v];
    r.dd = doff[v + 1] - r.od;
    return r;
}

// Live entry for neighbour x in row r: returns the raw entry (flags) or 0 with
// found = false.
__device__ __forceinline__ bool row_find(const int32_t *col, const int32_t *dcol, const RowRef &r,
                                         uint32_t x, uint32_t &ent) {
    int64_t p = find_sorted(col, r.ob, r.ob + r.db, x);
    if (p >= 0) {
        ent = (uint32_t)col[p];
        return !(ent & DEAD);
    }
    if (r.dd > 0) {
        int64_t q = find_sorted(dcol, r.od, r.od + r.dd, x);
        if (q >= 0) {
            ent = (uint32_t)dcol[q];
            return !(ent & DEAD);
        }
    }
    return false;
}

// Fenced search of a long base row: every stride-th neighbour id of the row is
// copied to LDS once per work item (stride: the smallest power of two from
// TC_FSTRIDE_MIN that needs at most TC_FCAP fences); a probe searches those
// fences in LDS and then only the stride-entry segment they select in global
// memory.  Rows of at most TC_FMIN entries, or longer than TC_FCAP *
// TC_FSTRIDE_MAX, are searched whole.
constexpr int TC_FSTRIDE_MIN = 8;
constexpr int TC_FSTRIDE_MAX = 2048;
constexpr int TC_FCAP = 128;  // fences per wave (rows up to 262,144 entries are fenced)
constexpr int TC_FMIN = 128;

// Position of neighbour x in the base row [ob, ob + db) whose fences f[k] =
// id(col[ob + k * stride]), k < nf, are in LDS; -1 if absent.
__device__ __forceinline__ int64_t find_fenced(const int32_t *__restrict__ col, int64_t ob, int64_t db,
                                               int stride, const uint32_t *f, int nf, uint32_t x) {
    if (x < f[0]) return -1;
    int lo = 0, hi = nf - 1;  // the last k with f[k] <= x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (f[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    const int64_t s0 = ob + (int64_t)lo * stride;
    return find_sorted(col, s0, min(s0 + stride, ob + db), x);
}

// Work items: a changed edge's shorter row is cut into pieces of TC_CHUNK entries,
// so that an edge between two hubs (tens of thousands of common candidates) is
// spread over many waves instead of holding one wave for the whole launch.
constexpr int TC_CHUNK = 256;

// cnt[i] = pieces of changed edge i (0 when its shorter row is empty); cnt[ne] = 0.
__global__ void k_tc_items(int64_t ne, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                           const int64_t *__restrict__ off, const int64_t *__restrict__ doff, int64_t *cnt) {
    for (int64_t i = gtid(); i <= ne; i += gstride()) {
        if (i == ne) {
            cnt[i] = 0;
            continue;
        }
        const int32_t a = eu[i], b = ev[i];
        const int64_t ta = (off[a + 1] - off[a]) + (doff[a + 1] - doff[a]);
        const int64_t tb = (off[b + 1] - off[b]) + (doff[b + 1] - doff[b]);
        cnt[i] = (min(ta, tb) + TC_CHUNK - 1) / TC_CHUNK;
    }
}

// One wave per work item; lanes walk the item's piece of the smaller row and probe
// the larger one.  start = exclusive scan of the piece counts (start[ne] = total).
__global__ __launch_bounds__(256) void k_tc_delta(int64_t ne, const int32_t *eu, const int32_t *ev,
                                                  const int64_t *__restrict__ start,
                                                  const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ col,
                                                  const int64_t *__restrict__ doff,
                                                  const int32_t *__restrict__ dcol, int64_t *part) {
    __shared__ uint32_t s_fence[256 / WAVE][TC_FCAP];
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    uint32_t *f = s_fence[threadIdx.x / WAVE];
    uint64_t acc = 0, walked = 0, probes = 0;
    const int64_t items = start[ne];
    for (int64_t it = wave_global; it < items; it += nwaves) {
        // the edge of item it: start[i] <= it < start[i + 1], found by a 64-way
        // search (each lane probes one point, a ballot keeps the prefix at or below it)
        int64_t lo = 0, hi = ne;  // start[lo] <= it < start[hi]
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + WAVE - 1) / WAVE;
            const int64_t p = lo + (int64_t)(l + 1) * step;
            const uint64_t le = __ballot(p < hi && start[p] <= it);
            lo += (int64_t)__popcll(le) * step;
            hi = min(hi, lo + step);
        }
        const int64_t i = lo, piece = it - start[i];
        int32_t a = eu[i], b = ev[i];
        RowRef ra = row_ref(off, doff, a), rb = row_ref(off, doff, b);
        if (ra.db + ra.dd > rb.db + rb.dd) {
            RowRef t = ra; ra = rb; rb = t;
        }
        const int64_t j0 = piece * TC_CHUNK, j1 = min(ra.db + ra.dd, j0 + TC_CHUNK);
        int stride = TC_FSTRIDE_MIN;
        while ((int64_t)stride * TC_FCAP < rb.db && stride < TC_FSTRIDE_MAX) stride <<= 1;
        const int64_t nf64 = (rb.db + stride - 1) / stride;
        const bool fenced = j1 > j0 && rb.db > TC_FMIN && nf64 <= TC_FCAP;
        const int nf = fenced ? (int)nf64 : 0;
        if (fenced) {
            wave_sync();  // every lane is done with the previous edge's fences
            for (int k = l; k < nf; k += WAVE) f[k] = (uint32_t)col[rb.ob + (int64_t)k * stride] & ID_MASK;
            wave_sync();
        }
        // global reads of one probe: the whole binary search, or the segment's
        const int64_t seg = fenced ? stride : rb.db;
        const int depth = (seg > 0 ? 64 - __clzll((unsigned long long)seg) : 0) +
                          (rb.dd > 0 ? 64 - __clzll((unsigned long long)rb.dd) : 0);
        if (l == 0) {
            walked += (j1 - j0) + nf;
            probes += (j1 - j0) * depth;
        }
        for (int64_t j = j0 + l; j < j1; j += WAVE) {
            uint32_t e = j < ra.db ? (uint32_t)col[ra.ob + j] : (uint32_t)dcol[ra.od + (j - ra.db)];
            if (e & DEAD) continue;
            uint32_t c = e & ID_MASK;
            uint32_t e2;
            bool hit;
            if (fenced) {
                const int64_t p = find_fenced(col, rb.ob, rb.db, stride, f, nf, c);
                if (p >= 0) {
                    e2 = (uint32_t)col[p];
                    hit = !(e2 & DEAD);
                } else {
                    hit = false;
                    if (rb.dd > 0) {
                        const int64_t q = find_sorted(dcol, rb.od, rb.od + rb.dd, c);
                        if (q >= 0) {
                            e2 = (uint32_t)dcol[q];
                            hit = !(e2 & DEAD);
                        }
                    }
                }
            } else {
                hit = row_find(col, dcol, rb, c, e2);
            }
            if (!hit) continue;
            int k = 1 + ((e & MARK) ? 1 : 0) + ((e2 & MARK) ? 1 : 0);
            acc += (uint64_t)(6 / k);
        }
    }
    // per-block partials (no contended atomics; summed in block order by k_tc_sum)
    __shared__ uint64_t s_p[3][256 / WAVE];
    acc = wave_sum(acc);
    walked = wave_sum(walked);
    probes = wave_sum(probes);
    const int wv = threadIdx.x / WAVE;
    if (l == 0) {
        s_p[0][wv] = acc;
        s_p[1][wv] = walked;
        s_p[2][wv] = probes;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint64_t s = 0;
        for (int q = 0; q < (int)blockDim.x / WAVE; ++q) s += s_p[threadIdx.x][q];
        part[3 * (int64_t)blockIdx.x + threadIdx.x] = (int64_t)s;
    }
}

// Sum of the per-block partials (triangle weight, entries walked, search steps).
__global__ __launch_bounds__(1024) void k_tc_sum(const int64_t *part, int64_t nblocks, int64_t *out) {
    __shared__ int64_t s[3][1024 / WAVE];
    int64_t a0 = 0, a1 = 0, a2 = 0;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
        a0 += part[3 * b];
        a1 += part[3 * b + 1];
        a2 += part[3 * b + 2];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        s[0][wv] = a0;
        s[1][wv] = a1;
        s[2][wv] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int64_t a = 0;
        for (int q = 0; q < (int)blockDim.x / WAVE; ++q) a += s[threadIdx.x][q];
        out[threadIdx.x] = a;
    }
}

int tc_delta(dg_graph *g, const int32_t *eu, const int32_t *ev, int64_t ne, uint64_t *sum6, int64_t *entries) {
    *sum6 = 0;
    if (entries) *entries = 0;
    if (ne <= 0) return DG_OK;
    hipStream_t s = g->stream;
    Dir &F = g->fwd;
    DG_TRY(counters_clear(g));
    // four waves per block; 16,384 blocks measured faster than a resident-size grid
    int64_t blocks = std::min<int64_t>((ne + 3) / 4, 16384);
    DG_TRY(g->ws.bpart.ensure(3 * (size_t)blocks + 8));
    DG_TRY(g->ws.tcitems.ensure(2 * ((size_t)ne + 1)));
    int64_t *cnt = g->ws.tcitems.p, *start = g->ws.tcitems.p + ne + 1;
    hipLaunchKernelGGL(k_tc_items, dim3(grid_for(ne + 1)), dim3(256), 0, s, ne, eu, ev, F.off.p, F.doff.p, cnt);
    DG_HIP(hipGetLastError());
    DG_TRY(scan_excl(g, cnt, start, ne + 1));
    int ps = prof_begin("tc_delta", s);
    hipLaunchKernelGGL(k_tc_delta, dim3((unsigned)blocks), dim3(256), 0, s, ne, eu, ev, start, F.off.p, F.col.p,
                       F.doff.p, F.dcol.p, g->ws.bpart.p);
    prof_end(ps, s, 0.0);
    // counters C_AUX1, C_AUX2, C_AUX3 = 6 x changed triangles, entries walked, search steps
    static_assert(C_AUX2 == C_AUX1 + 1 && C_AUX3 == C_AUX1 + 2, "three consecutive counters");
    hipLaunchKernelGGL(k_tc_sum, dim3(1), dim3(1024), 0, s, g->ws.bpart.p, blocks, g->ws.dcnt + C_AUX1);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    *sum6 = (uint64_t)g->ws.hcnt[C_AUX1];
    if (entries) *entries = g->ws.hcnt[C_AUX2];  // shorter-row entries intersected
    // per changed edge its endpoints' offsets (32 B); per entry of the shorter row
    // and per fence of a long row 4 B; per global search step into the longer row
    // (the whole row, or the segment a fence search selects) 4 B
    prof_add(ps, 32.0 * (double)ne + 4.0 * (double)g->ws.hcnt[C_AUX2] + 4.0 * (double)g->ws.hcnt[C_AUX3]);
    return DG_OK;
}

// ---- static count on a merged (plain CSR) graph -------------------------------------

__device__ __forceinline__ bool rank_lt(int32_t du, int32_t u, int32_t dv, int32_t v) {
    return du < dv || (du == dv && u < v);
}

// Forward (oriented) lists: N+(x) = the neighbours of x ranked above x, kept in id
// order.  One wave per row; pass 1 writes |N+(x)| to odeg, pass 2 fills ocol
// from the scanned offsets ooff (ballot compaction keeps the order).
template <bool FILL>
__global__ __launch_bounds__(256) void k_tc_orient(int32_t n, const int64_t *__restrict__ off,
                                                   const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ deg, int64_t *odeg,
                                                   const int64_t *__restrict__ ooff, int32_t *ocol) {
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    for (int64_t x = wave_global; x < n; x += nwaves) {
        const int64_t xs = off[x], xe = off[x + 1];
        const int32_t dx = deg[x];
        int64_t cnt = 0;
        const int64_t base = FILL ? ooff[x] : 0;
        for (int64_t j0 = xs; j0 < xe; j0 += WAVE) {
            const int64_t j = j0 + l;
            bool up = false;
            int32_t y = 0;
            if (j < xe) {
                const uint32_t c = (uint32_t)col[j];
                y = (int32_t)(c & ID_MASK);
                up = !(c & DEAD) && rank_lt(dx, (int32_t)x, deg[y], y);
            }
            const uint64_t b = ballot(up);
            if (FILL && up) ocol[base + cnt + __popcll(b & lanemask_lt())] = y;
            cnt += __popcll(b);
        }
        if (!FILL && l == 0) odeg[x] = cnt;
    }
}

// Every triangle, ranked a < b < c, is counted once: at x = a and y = b, as the
// common element c of N+(a) and N+(b).  One wave per row x copies N+(x) to LDS
// (when it fits) and walks y over N+(x).  For each y the lanes either stream
// N+(y) and binary-search the LDS copy (one coalesced load per 64 elements), or,
// when N+(y) is much longer, take the elements of N+(x) and binary-search N+(y)
// in memory.
constexpr int TCF_CAP = 1024;  // forward-list entries of a row staged in LDS, per wave

__device__ __forceinline__ bool lds_has(const int32_t *a, int len, int32_t v) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < len && a[lo] == v;
}

__global__ __launch_bounds__(256) void k_tc_forward(int32_t n, const int64_t *__restrict__ ooff,
                                                    const int32_t *__restrict__ ocol,
                                                    unsigned long long *total) {
    __shared__ int32_t s_nx[256 / WAVE][TCF_CAP];
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    int32_t *sx = s_nx[threadIdx.x / WAVE];
    uint64_t acc = 0;
    for (int64_t x = wave_global; x < n; x += nwaves) {
        const int64_t xs = ooff[x], xe = ooff[x + 1];
        const int64_t dx = xe - xs;
        if (dx < 2) continue;
        const bool staged = dx <= TCF_CAP;
        if (staged) {
            for (int64_t j = l; j < dx; j += WAVE) sx[j] = ocol[xs + j];
            wave_sync();
        }
        const int64_t rx = (dx + WAVE - 1) / WAVE;
        for (int64_t p0 = 0; p0 < dx; p0 += WAVE) {
            // lane k fetches the list bounds of the k-th y of this chunk of N+(x)
            int64_t mys = 0, mye = 0;
            if (p0 + l < dx) {
                const int32_t y = staged ? sx[p0 + l] : ocol[xs + p0 + l];
                mys = ooff[y];
                mye = ooff[y + 1];
            }
            const int cnt = (int)(dx - p0 < WAVE ? dx - p0 : WAVE);
            for (int k = 0; k < cnt; ++k) {
                const int64_t ys = __shfl(mys, k, WAVE), ye = __shfl(mye, k, WAVE);
                const int64_t dy = ye - ys;
                if (staged && (dy + WAVE - 1) / WAVE <= 4 * rx) {
                    // four loads in flight per lane before the LDS searches
                    for (int64_t j0 = ys + l; j0 < ye; j0 += 4 * WAVE) {
                        int32_t v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = j0 + u * WAVE < ye ? ocol[j0 + u * WAVE] : -1;
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (v[u] >= 0 && lds_has(sx, (int)dx, v[u])) ++acc;
                    }
                } else {
                    for (int64_t j = xs + l; j < xe; j += WAVE)
                        if (find_sorted(ocol, ys, ye, (uint32_t)ocol[j]) >= 0) ++acc;
                }
            }
        }
        if (staged) wave_sync();  // the next row overwrites the staging
    }
    acc = wave_sum(acc);
    if (l == 0 && acc) atomicAdd(total, (unsigned long long)acc);
}

int tc_count_static(dg_graph *g, uint64_t *count) {
    DG_TRY(graph_merge(g));
    hipStream_t s = g->stream;
    Dir &F = g->fwd;
    const int32_t n = g->n;
    // the merge's spare target buffers hold the oriented lists (m / 2 entries)
    DG_TRY(F.off2.ensure((size_t)n + 1));
    DG_TRY(F.col2.ensure((size_t)(F.m / 2) + 1));
    DG_TRY(g->ws.scan64.ensure((size_t)n + 1));
    int64_t *odeg = g->ws.scan64.p, *ooff = F.off2.p;
    int32_t *ocol = F.col2.p;
    const int blocks = (int)std::min<int64_t>(((int64_t)n + 3) / 4, 32768);
    hipLaunchKernelGGL(k_tc_orient<false>, dim3(blocks), dim3(256), 0, s, n, F.off.p, F.col.p, F.deg.p, odeg,
                       nullptr, nullptr);
    DG_TRY(fill_i64(odeg + n, 0, 1, s));
    DG_TRY(scan_excl(g, odeg, ooff, (int64_t)n + 1));
    hipLaunchKernelGGL(k_tc_orient<true>, dim3(blocks), dim3(256), 0, s, n, F.off.p, F.col.p, F.deg.p, nullptr,
                       ooff, ocol);
    DG_TRY(counters_clear(g));
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(g->ws.dcnt + C_TC1);
    hipLaunchKernelGGL(k_tc_forward, dim3(blocks), dim3(256), 0, s, n, ooff, ocol, acc);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    *count = (uint64_t)g->ws.hcnt[C_TC1];
    return DG_OK;
}

}  // namespace dg
