/*
 * CPU oracle for the dynamic-graph hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no code, header or constant with the GPU library.
 *
 * What it computes is the definition the dynamic method must reach: apply an
 * update batch to an edge set, then recompute the property statically on the
 * updated graph.  The dynamic algorithms of the paper (Appendix A listings for
 * dynamic SSSP, PR and TC) all claim to produce exactly the static result on the
 * updated graph G' (Section 3.1: only the affected part is recomputed, the result
 * is the same), so the static recomputation is the oracle:
 *
 *   orc_apply     -- G' = (E \ D) U A under the batch rules listed at the function
 *   orc_sssp      -- Dijkstra with a binary heap and 64-bit sums
 *   orc_pagerank  -- FP64 power iteration (dangling mass spread uniformly), L1 stop
 *   orc_tc        -- exact triangle count, node iterator u < v < w (Appendix A,
 *                    staticTC) with a merge intersection of sorted rows
 *   orc_symmetrise-- the undirected view {u,v} of a directed edge set
 *
 * Plain, single-threaded C with qsort; nothing is blocked, fused or reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF 1073741823 /* INT_MAX / 2: the paper's INF for unreachable vertices */
#define ORC_WMAX (1 << 30) /* weights must lie in [1, 2^30) */

typedef struct {
    int64_t key; /* (u << 32) | v */
    int32_t w;
} orc_kw;

static int cmp_kw(const void *a, const void *b) {
    const orc_kw *x = (const orc_kw *)a, *y = (const orc_kw *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return 0;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y);
}

static int64_t make_key(int32_t u, int32_t v, int undirected) {
    if (undirected && u > v) { int32_t t = u; u = v; v = t; }
    return ((int64_t)u << 32) | (int64_t)(uint32_t)v;
}

/* index of key in sorted a[0..n) or -1 */
static int64_t find_i64(const int64_t *a, int64_t n, int64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo] == key) ? lo : -1;
}

static int64_t find_kw(const orc_kw *a, int64_t n, int64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid].key < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo].key == key) ? lo : -1;
}

/*
 * Apply one batch of edge updates to a simple graph (Section 3.3.1 Batch,
 * Section 3.3.2 OnAdd/OnDelete; the drivers of Appendix A delete before they add).
 * Rules, in the readings of the silent points:
 *   B1  G' = (E \ D) U A: deletions are applied before insertions.
 *   B2  inserting an edge that is present in E \ D changes nothing (counted as
 *       an ignored insert; the old weight stays).
 *   B3  deleting an absent edge changes nothing (ignored delete).
 *   B4  several inserts of one edge in a batch: the smallest weight wins.
 *   B5  an edge deleted and inserted in one batch ends present with the new weight.
 *   B6  a self-loop or a vertex id outside [0, n) anywhere in the batch rejects the
 *       whole batch (return -1, nothing written); so does an op other than 0/1 or an
 *       insert weight outside [1, 2^30) (weights are positive).
 *   B7  undirected graphs: every edge and every update is an unordered pair.
 *   B8  the weight field of a deletion is ignored.
 * Output: G' sorted by (u, v) (u < v for undirected).  stats[0..3] = deletions
 * applied, insertions applied, ignored deletions, ignored insertions (duplicates
 * inside the batch are not counted).  Returns |E'|, -1 on an invalid batch, -2 on an
 * input graph that is not simple, -3 if cap is too small.
 */
int64_t orc_apply(int32_t n, int32_t undirected, int64_t m, const int32_t *src,
                  const int32_t *dst, const int32_t *w, int64_t k, const int32_t *bsrc,
                  const int32_t *bdst, const int32_t *bw, const uint8_t *bop, int32_t *osrc,
                  int32_t *odst, int32_t *ow, int64_t cap, int64_t *stats) {
    for (int64_t i = 0; i < k; ++i) {
        if (bsrc[i] < 0 || bsrc[i] >= n || bdst[i] < 0 || bdst[i] >= n) return -1;
        if (bsrc[i] == bdst[i]) return -1;
        if (bop[i] > 1) return -1;
        if (bop[i] == 1 && (bw[i] < 1 || bw[i] >= ORC_WMAX)) return -1;
    }
    orc_kw *E = (orc_kw *)malloc(sizeof(orc_kw) * (m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        E[i].key = make_key(src[i], dst[i], undirected);
        E[i].w = w ? w[i] : 1;
    }
    qsort(E, (size_t)m, sizeof(orc_kw), cmp_kw);
    for (int64_t i = 1; i < m; ++i)
        if (E[i].key == E[i - 1].key) { free(E); return -2; }

    int64_t nd = 0, na = 0;
    for (int64_t i = 0; i < k; ++i) (bop[i] == 0) ? ++nd : ++na;
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (nd > 0 ? nd : 1));
    orc_kw *A = (orc_kw *)malloc(sizeof(orc_kw) * (na > 0 ? na : 1));
    nd = na = 0;
    for (int64_t i = 0; i < k; ++i) {
        int64_t key = make_key(bsrc[i], bdst[i], undirected);
        if (bop[i] == 0) D[nd++] = key;
        else { A[na].key = key; A[na].w = bw[i]; ++na; }
    }
    qsort(D, (size_t)nd, sizeof(int64_t), cmp_i64);
    qsort(A, (size_t)na, sizeof(orc_kw), cmp_kw);
    /* distinct deletions; distinct insertions keeping the first = smallest weight (B4) */
    int64_t ndu = 0;
    for (int64_t i = 0; i < nd; ++i)
        if (ndu == 0 || D[ndu - 1] != D[i]) D[ndu++] = D[i];
    int64_t nau = 0;
    for (int64_t i = 0; i < na; ++i)
        if (nau == 0 || A[nau - 1].key != A[i].key) A[nau++] = A[i];

    /* E1 = E \ D */
    orc_kw *E1 = (orc_kw *)malloc(sizeof(orc_kw) * (m > 0 ? m : 1));
    int64_t m1 = 0, deleted = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (find_i64(D, ndu, E[i].key) >= 0) ++deleted;
        else E1[m1++] = E[i];
    }
    /* G' = E1 U (A \ E1) as a sorted merge */
    int64_t inserted = 0, ign_ins = 0, out = 0, j = 0;
    for (int64_t i = 0; i < nau; ++i) {
        if (find_kw(E1, m1, A[i].key) >= 0) { ++ign_ins; continue; }
        while (j < m1 && E1[j].key < A[i].key) {
            if (out >= cap) goto overflow;
            osrc[out] = (int32_t)(E1[j].key >> 32); odst[out] = (int32_t)(E1[j].key & 0xffffffff);
            ow[out] = E1[j].w; ++out; ++j;
        }
        if (out >= cap) goto overflow;
        osrc[out] = (int32_t)(A[i].key >> 32); odst[out] = (int32_t)(A[i].key & 0xffffffff);
        ow[out] = A[i].w; ++out; ++inserted;
    }
    while (j < m1) {
        if (out >= cap) goto overflow;
        osrc[out] = (int32_t)(E1[j].key >> 32); odst[out] = (int32_t)(E1[j].key & 0xffffffff);
        ow[out] = E1[j].w; ++out; ++j;
    }
    if (stats) {
        stats[0] = deleted; stats[1] = inserted;
        stats[2] = ndu - deleted; stats[3] = ign_ins;
    }
    free(E); free(D); free(A); free(E1);
    return out;
overflow:
    free(E); free(D); free(A); free(E1);
    return -3;
}

/* Out-adjacency in CSR form by a counting sort (rows keep the input order). */
static void build_out_csr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          int64_t **off_out, int32_t **col_out, int64_t **eid_out) {
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
    int64_t *eid = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) off[src[i] + 1]++;
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m; ++i) {
        int64_t p = fill[src[i]]++;
        col[p] = dst[i];
        eid[p] = i;
    }
    free(fill);
    *off_out = off; *col_out = col; *eid_out = eid;
}

/* ---- Dijkstra --------------------------------------------------------------- */

typedef struct { int64_t d; int32_t v; } orc_heap_item;

static void heap_push(orc_heap_item *h, int64_t *len, int64_t d, int32_t v) {
    int64_t i = (*len)++;
    h[i].d = d; h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        orc_heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static orc_heap_item heap_pop(orc_heap_item *h, int64_t *len) {
    orc_heap_item top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *len && h[l].d < h[s].d) s = l;
        if (r < *len && h[r].d < h[s].d) s = r;
        if (s == i) break;
        orc_heap_item t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

/*
 * Single-source shortest distances on G (directed arcs src->dst, weight w):
 * what staticSSSP of Appendix A computes with its Bellman-Ford style fixed point,
 * here by Dijkstra with lazy deletion.  dist[v] = INF (2^30 - 1) when v is
 * unreachable.  Returns 0, -1 on a bad source, -2 if a finite distance reaches INF.
 */
int orc_sssp(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *w,
             int32_t source, int32_t *dist) {
    if (source < 0 || source >= n) return -1;
    int64_t *off; int32_t *col; int64_t *eid;
    build_out_csr(n, m, src, dst, &off, &col, &eid);
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    char *done = (char *)calloc((size_t)n, 1);
    for (int32_t v = 0; v < n; ++v) d[v] = INT64_MAX;
    orc_heap_item *h = (orc_heap_item *)malloc(sizeof(orc_heap_item) * (size_t)(m + 2));
    int64_t len = 0;
    d[source] = 0;
    heap_push(h, &len, 0, source);
    while (len > 0) {
        orc_heap_item it = heap_pop(h, &len);
        if (done[it.v]) continue;
        done[it.v] = 1;
        for (int64_t p = off[it.v]; p < off[it.v + 1]; ++p) {
            int32_t x = col[p];
            int64_t cand = it.d + (int64_t)w[eid[p]];
            if (cand < d[x]) { d[x] = cand; heap_push(h, &len, cand, x); }
        }
    }
    int rc = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (d[v] == INT64_MAX) dist[v] = ORC_INF;
        else if (d[v] >= ORC_INF) { dist[v] = ORC_INF; rc = -2; }
        else dist[v] = (int32_t)d[v];
    }
    free(off); free(col); free(eid); free(d); free(done); free(h);
    return rc;
}

/* ---- PageRank -------------------------------------------------------------- */

/*
 * PageRank by FP64 power iteration (Appendix A, staticPR: Jacobi steps from
 * 1/N with damping delta).  The listing drops the rank held by vertices without
 * out-edges; here it is spread uniformly, the standard definition, so the ranks
 * sum to one:
 *   pi_0 = 1/n,
 *   pi_{k+1}[v] = (1-d)/n + d * ( sum_{u->v} pi_k[u]/outdeg(u) + D_k/n ),
 *   D_k = sum of pi_k[u] over u with outdeg(u) = 0,
 * stopping after the first step with ||pi_{k+1} - pi_k||_1 <= tol, or after
 * max_iter steps.  *iters receives the number of steps.  Returns 0 if converged,
 * 1 if max_iter was reached, -1 on bad arguments.
 */
int orc_pagerank(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, double d,
                 double tol, int32_t max_iter, double *rank, int32_t *iters) {
    if (n <= 0 || max_iter < 1) return -1;
    int64_t *outdeg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) outdeg[src[i]]++;
    double *pi = (double *)malloc(sizeof(double) * (size_t)n);
    double *acc = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) pi[v] = 1.0 / n;
    int32_t it = 0;
    int rc = 1;
    while (it < max_iter) {
        double dang = 0.0;
        for (int32_t u = 0; u < n; ++u)
            if (outdeg[u] == 0) dang += pi[u];
        for (int32_t v = 0; v < n; ++v) acc[v] = 0.0;
        for (int64_t i = 0; i < m; ++i) acc[dst[i]] += pi[src[i]] / (double)outdeg[src[i]];
        double diff = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            double val = (1.0 - d) / n + d * (acc[v] + dang / n);
            diff += fabs(val - pi[v]);
            pi[v] = val;
        }
        ++it;
        if (diff <= tol) { rc = 0; break; }
    }
    memcpy(rank, pi, sizeof(double) * (size_t)n);
    if (iters) *iters = it;
    free(outdeg); free(pi); free(acc);
    return rc;
}

/* ---- Triangle counting ------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/*
 * Number of triangles of a simple undirected graph given as m unordered pairs
 * (each edge once, either orientation).  Every triangle {a < b < c} is counted
 * exactly once: for every vertex a, for every neighbour b > a, the common
 * neighbours c > b of a and b (Appendix A, staticTC, which enumerates u < v < w
 * around the middle vertex; the same set of triples).  Returns 0, -1 on bad input.
 */
int orc_tc(int32_t n, int64_t m, const int32_t *u, const int32_t *v, uint64_t *count) {
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n || u[i] == v[i]) { free(off); return -1; }
        off[u[i] + 1]++; off[v[i] + 1]++;
    }
    for (int32_t x = 0; x < n; ++x) off[x + 1] += off[x];
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m; ++i) {
        col[fill[u[i]]++] = v[i];
        col[fill[v[i]]++] = u[i];
    }
    free(fill);
    for (int32_t x = 0; x < n; ++x)
        qsort(col + off[x], (size_t)(off[x + 1] - off[x]), sizeof(int32_t), cmp_i32);
    uint64_t total = 0;
    for (int32_t a = 0; a < n; ++a) {
        for (int64_t p = off[a]; p < off[a + 1]; ++p) {
            int32_t b = col[p];
            if (b <= a) continue;
            /* common neighbours c > b of a and b */
            int64_t i = off[a], j = off[b];
            while (i < off[a + 1] && j < off[b + 1]) {
                if (col[i] < col[j]) ++i;
                else if (col[i] > col[j]) ++j;
                else { if (col[i] > b) ++total; ++i; ++j; }
            }
        }
    }
    *count = total;
    free(off); free(col);
    return 0;
}

/*
 * Undirected view of a directed edge set: {u, v} is an edge iff (u, v) or (v, u)
 * is an arc.  Writes each edge once as (min, max), sorted; returns the count.
 */
int64_t orc_symmetrise(int64_t m, const int32_t *src, const int32_t *dst, int32_t *ou,
                       int32_t *ov) {
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) keys[i] = make_key(src[i], dst[i], 1);
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t c = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (c > 0 && keys[i] == ((int64_t)ou[c - 1] << 32 | (uint32_t)ov[c - 1])) continue;
        ou[c] = (int32_t)(keys[i] >> 32);
        ov[c] = (int32_t)(keys[i] & 0xffffffff);
        ++c;
    }
    free(keys);
    return c;
}
