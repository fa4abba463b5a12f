/*
 * dg.h -- C ABI of the MI355X dynamic-graph library.
 *
 * The operations follow the problem statement of Kumar et al., "Generating
 * Dynamic Graph Algorithms for Multiple Backends for a Graph DSL" (arXiv
 * 2507.11094): given a graph G and a batch of edge insertions and deletions
 * (Delta G), update G and recompute only what the batch disturbs.  The three
 * maintained properties are those of the paper's Appendix A programs:
 * single-source shortest paths (DynSSSP), PageRank (DynPR) and triangle count
 * (DynTC).  The graph store is the diff-CSR of Section 3.5: a sorted CSR whose
 * deleted entries carry a tombstone, one sorted diff level for insertions, and a
 * merge back into plain CSR once the diff and tombstones pass a threshold.
 *
 * Conventions for every call:
 *   - Return value: DG_OK (0) or a negative DG_E* code.  dg_last_error() gives a
 *     message for the calling thread's last failure.
 *   - Vertex ids are int32 in [0, n) with n <= 2^30; edge weights are int32 in
 *     [1, 2^30) (positive, so a shortest-path parent is always strictly closer to
 *     the source).  Graphs are simple: no self-loops, no parallel edges.
 *   - Pointer arguments are host memory unless DG_DEVICE_PTRS is passed in the
 *     call's flags, in which case they are device memory of the current HIP
 *     device.  The library copies what it needs and never keeps a caller pointer.
 *   - All device memory behind a handle is owned by the library and released by
 *     the matching destroy/detach call.
 *   - Work is issued on the graph's stream (dg_graph_set_stream; default: the
 *     null stream).  Calls return after their results are complete, except where
 *     a call says otherwise.  One host thread at a time may use a given graph;
 *     different graphs are independent.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------ */
#define DG_OK 0
#define DG_EINVAL (-1)   /* bad argument or invalid batch; nothing was changed     */
#define DG_ENOMEM (-2)   /* device allocation failed; nothing was changed           */
#define DG_EDEVICE (-3)  /* a HIP runtime call failed                               */
#define DG_ESTATE (-4)   /* handle unusable (earlier device error) or wrong kind    */
#define DG_EBUSY (-5)    /* server queue full                                       */
#define DG_EBUDGET (-6)  /* request exceeds the server's memory budget              */
#define DG_ENOTFOUND (-7)/* no such request / result not ready                      */

/* Distance of a vertex the source cannot reach: INT_MAX / 2, the paper's INF
 * (Appendix A, Dynamic SSSP listing).  Distances saturate: a vertex whose
 * shortest distance is DG_INF or more is reported as DG_INF with parent -1, like
 * an unreachable one, and every other vertex keeps its exact distance. */
#define DG_INF 1073741823

/* ---- flags --------------------------------------------------------------------- */
#define DG_DIRECTED 0u
#define DG_UNDIRECTED 1u     /* graph_create: each edge given once, stored both ways */
#define DG_DEVICE_PTRS 2u    /* pointer arguments of this call are device memory     */
#define DG_INCREMENTAL 4u    /* apply_batch: every update is an insertion (op may be NULL) */
#define DG_DECREMENTAL 8u    /* apply_batch: every update is a deletion (op may be NULL)   */

typedef struct dg_graph dg_graph;
typedef struct dg_query dg_query;
typedef struct dg_snapshot dg_snapshot;

/* Tunables.  Zero-initialise and set what you need; zero fields take defaults. */
typedef struct dg_config {
    /* Merge the diff level and tombstones back into plain CSR when
     * (diff entries + tombstones) > merge_threshold * (live edges)
     * (Section 3.5: the chain of diffs is merged after a configurable number of
     * batches).  Default 0.05.  A negative value merges after every batch. */
    double merge_threshold;
    /* PageRank stops when the L1 step is <= tol * pr_tol_scale.  Default 1. */
    double pr_tol_scale;
    /* Vertices with more edges than this are split into chunks across waves.
     * Default 0 = autotuned table / built-in value.  While no row is longer (the
     * library keeps an upper bound on the longest row), the host-driven frontier
     * steps launch no chunk kernel at all. */
    int32_t heavy_degree;
    /* Workgroups of the persistent SSSP kernel; 0 = autotuned / built-in. */
    int32_t persistent_groups;
    /* SSSP update schedule (Appendix A, Dynamic SSSP: cut, pull, push to a fixed
     * point): 0 (default) or 3 = frontier steps launched one at a time from the
     * host with grids sized to each frontier, the host reading every step's count;
     * 2 = frontier steps with device-side counts and termination: the steps
     * (near-far rounds too, with the bucket threshold and the far pile on the
     * device) are captured once into hipGraphs and replayed per batch, and the host
     * reads the counts once per replay of 8-16 steps instead of once per step (the
     * default for graph sets; on single graphs measured no faster, the replayed
     * graph nodes costing more than the round trips they save); 1 = persistent
     * work-queue kernels (one launch per phase).  Same results; the static solve
     * at attach uses host-driven frontier steps unless 1. */
    int32_t sssp_persistent;
    /* PageRank iteration after a batch: 0 = automatic (global dangling-uniform
     * form when the affected set holds >= 20% of the edges, else the local
     * restricted form), 1 = always local, 2 = always global, 3 = residual push
     * (the in-place alternative the paper's evaluation discusses): every vertex
     * keeps the residual of the local system, a batch recomputes it where an
     * equation changed, and rounds push every vertex whose residual exceeds
     * tol * sum(x) / (4 n) to its out-neighbours until none does.  Same ranks
     * within the tolerance; work stays near the batch where the residual fades
     * before it spreads (long paths, few dangling vertices); last bits vary run
     * to run (FP64 atomics). */
    int32_t pr_mode;
    /* Whole-graph PageRank pull (static solve and the global form): 0 = merge-path
     * tiles (equal rows + entries per workgroup; column and offset streams read
     * with non-temporal hints so they do not evict the gathered values from L2;
     * default), 1 = the per-vertex wave kernel that the affected-set iteration
     * uses, 2 = merge-path tiles without the hints.  Same results up to rounding
     * (0 and 2: bit-identical). */
    int32_t pr_pull;
    /* Frontier-step SSSP schedule: 0 = plain Bellman-Ford rounds (default);
     * > 0 = near-far buckets of this width (vertices at distance >= the current
     * threshold wait in a far pile until the nearer ones settle), which cuts the
     * re-relaxations of high-diameter graphs such as road networks.  Same result. */
    int32_t sssp_delta;
    /* > 0: also merge after this many batches since the last merge (Section 3.5
     * merges after a configurable number of batches); 0 = threshold only. */
    int32_t merge_period;
    /* Rows + entries per merge-path tile of the whole-graph pull: 1024, 2048 or
     * 4096 (0 or anything else: 2048). */
    int32_t pr_tile;
    /* Rows + entries per merge-path tile of the CSR merge: 512, 1024 or 2048
     * (0 or anything else: 2048). */
    int32_t merge_tile;
    /* Vertex order inside the library (dg_graph_create only; sets keep the order
     * given): 0 = by degree, highest first, so that the hot rows and the values
     * gathered from them share cache lines; 1 = as given.  Every id the caller
     * passes or reads back is the caller's own either way. */
    int32_t vertex_order;
    /* Placement of a new edge (Section "Modified Graph Representation: diff-CSR"):
     * 0 = in a tombstoned slot of its row when one lies next to its sorted
     * position (the row stays sorted; among new edges wanting one slot, the
     * smallest takes it), else in the diff level (default); 1 = always in the diff
     * level (a slot of the same edge is still revived). */
    int32_t diff_only;
    /* Jacobi PageRank steps: 0 = plain steps, as in the Appendix A listings
     * (default); 1 = extrapolated steps: when two successive step vectors are
     * parallel (a least-squares fit s_k = lam s_{k-1} leaves at most 5 % of s_k
     * unexplained, 0 < lam <= 0.9), the error is dominated by one eigenvector and
     * the next step also moves lam / (1 - lam) times its own length further, which
     * removes that component (Aitken's process along the step).  Bipartite graphs
     * such as grids carry their error in pairs of modes near +d and -d, whose
     * successive steps never line up; there a fit of s_k against s_{k-2}
     * (mu = lam^2, at most 15 % unexplained, 0 < mu <= 0.81) moves the two-step
     * map instead, along the sum of the last two steps.  Convergence is still
     * declared only on a plain step, so the stopping rule bounds the error as in
     * plain Jacobi; the ranks differ from the plain iterates within that bound
     * (they are usually closer to the fixed point).  The fits keep the previous
     * step in n floats (4 bytes read and written per vertex and step), and the one
     * before it in n more floats only once four plain steps without a move have
     * passed and the one-step fit explains at most 5 % of |s_k|^2 (orthogonal
     * successive steps, as on grids).  They stop after 24 plain steps without a
     * move or once the step is too small for any move. */
    int32_t pr_extrapolate;
} dg_config;

/* Per-batch statistics and phase timings (HIP events on the graph's stream). */
typedef struct dg_batch_stats {
    int64_t updates;            /* updates in the call                                  */
    int64_t deleted;            /* edges removed (undirected: counted once per edge)    */
    int64_t inserted;           /* edges added, including re-inserts of deleted edges   */
    int64_t ignored_del;        /* deletions of absent edges                            */
    int64_t ignored_ins;        /* insertions of present edges                          */
    int64_t diff_entries;       /* diff-level entries after the call                    */
    int64_t tombstones;         /* tombstoned entries after the call                    */
    int32_t merged;             /* merges performed                                     */
    int32_t chunks;             /* batch_size chunks processed                          */
    int64_t sssp_invalidated;   /* vertices whose tree path was cut                     */
    int64_t sssp_relaxed;       /* vertices processed by push relaxation                */
    int32_t sssp_steps;         /* frontier steps                                       */
    int32_t pr_iterations;      /* Jacobi iterations                                    */
    int64_t pr_affected;        /* vertices in the affected set                         */
    int64_t edges_traversed;    /* adjacency entries examined: PageRank pulls (entries x steps), the
                                   SSSP rounds (entries of the rows each cut, pull and push step
                                   walks) and the triangle kernel's intersections */
    int64_t tc_removed;         /* triangles removed by the deletions                   */
    int64_t tc_added;           /* triangles added by the insertions                    */
    float t_validate_ms, t_update_ms, t_merge_ms, t_sssp_ms, t_pr_ms, t_tc_ms, t_total_ms;
    int32_t pr_moves;           /* extrapolation moves of the PageRank steps            */
} dg_batch_stats;

const char *dg_last_error(void);

/* Device allocator hook for all library allocations (default hipMalloc/hipFree).
 * Must be set before any graph exists; alloc returns NULL on failure. */
int dg_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*free_fn)(void *p, void *ctx),
                     void *ctx);

/* ---- graph ----------------------------------------------------------------------- */

/* Build a device-resident graph from an edge list (CSR and reverse CSR, Section
 * 3.5 "diff-CSR" with an empty diff level).  src/dst/w hold m entries; w may be
 * NULL (all weights 1).  Directed: m arcs src->dst.  DG_UNDIRECTED: m unordered
 * pairs, each stored in both directions.  Duplicate edges or self-loops, ids
 * outside [0, n), or weights outside [1, 2^30) give DG_EINVAL.  flags may add
 * DG_DEVICE_PTRS.  cfg may be NULL. */
int dg_graph_create(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    const int32_t *w, uint32_t flags, const dg_config *cfg, dg_graph **out);
int dg_graph_destroy(dg_graph *g);

/* Issue the graph's work on this hipStream_t (NULL = null stream). */
int dg_graph_set_stream(dg_graph *g, void *hip_stream);

/* n, live edge count (undirected: edges, not arcs), diff-level entries and
 * tombstones of the forward direction.  Any output pointer may be NULL. */
int dg_graph_info(dg_graph *g, int32_t *n, int64_t *m_live, int64_t *diff_entries,
                  int64_t *tombstones);

/* Copy the live edge set to host arrays, sorted by (src, dst); undirected graphs
 * give each edge once with src < dst.  Call with src == NULL to get *m only;
 * otherwise *m must hold the capacity on entry and receives the count. */
int dg_graph_export(dg_graph *g, int64_t *m, int32_t *src, int32_t *dst, int32_t *w);

/* Merge diff level and tombstones into plain CSR now (Section 3.5). */
int dg_graph_merge(dg_graph *g);

/* Apply k updates (updateCSRDel then updateCSRAdd, Section 3.2 and the
 * Appendix A drivers), in chunks of batch_size (<= 0: one chunk), as the Batch
 * construct of Section 3.3.1 does, and update every attached query after each
 * chunk.  op[i] = 0 deletes src[i]->dst[i] (w[i] ignored), op[i] = 1 inserts
 * it with weight w[i] (w may be NULL: weight 1).  Semantics per chunk:
 * G' = (E \ D) U A; deleting an absent edge or inserting a present one changes
 * nothing; repeated inserts of one edge keep the smallest weight; an edge both
 * deleted and inserted ends present with the inserted weight.  Undirected graphs
 * take unordered pairs.  A self-loop, an id outside [0, n), an op other than 0/1
 * or a weight outside [1, 2^30) anywhere in a chunk rejects that chunk with
 * DG_EINVAL before any change (earlier chunks stay applied).  flags may hold
 * DG_DEVICE_PTRS and one of DG_INCREMENTAL / DG_DECREMENTAL (the paper's
 * partially dynamic cases, Section 3.2: only additions or only deletions); with
 * a mode op may be NULL, and an op that differs from the mode rejects the chunk.
 * stats may be NULL. */
int dg_apply_batch(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst,
                   const int32_t *w, const uint8_t *op, int64_t batch_size, uint32_t flags,
                   dg_batch_stats *stats);

/* Device-side copy of the graph and all attached query state, and its restore
 * (for repeated timing of the same batch on the same graph). */
int dg_snapshot_save(dg_graph *g, dg_snapshot **out);
int dg_snapshot_restore(dg_graph *g, const dg_snapshot *s);
int dg_snapshot_free(dg_snapshot *s);

/* ---- maintained queries -------------------------------------------------------- */

/* Attach a shortest-path query from `source`: computes the static solution
 * (staticSSSP of Appendix A) and keeps it exact across dg_apply_batch calls
 * (OnDelete / Decremental / OnAdd / Incremental of the Dynamic SSSP listing). */
int dg_sssp_attach(dg_graph *g, int32_t source, dg_query **q);

/* Attach PageRank with damping in (0, 1), L1 tolerance tol > 0 and an iteration
 * cap (staticPR of Appendix A, with delta = damping and beta = tol); kept current
 * across batches by the Incremental/Decremental PR steps on the affected set. */
int dg_pr_attach(dg_graph *g, double damping, double tol, int32_t max_iter, dg_query **q);

/* Attach a triangle count (staticTC, then the Decremental/Incremental TC steps
 * of Appendix A).  Undirected graphs only (DG_EINVAL otherwise). */
int dg_tc_attach(dg_graph *g, dg_query **q);

int dg_query_detach(dg_query *q);

/* Distances (DG_INF when unreachable) and one shortest-path tree (parent -1 for
 * the source and unreachable vertices); n entries each.  parent may be NULL. */
int dg_sssp_read(dg_query *q, int32_t *dist, int32_t *parent, uint32_t flags);

/* PageRank normalised to sum 1 (n entries); iters (nullable) receives the
 * iterations of the last solve, converged (nullable) 1 if it met the tolerance. */
int dg_pr_read(dg_query *q, double *rank, int32_t *iters, int32_t *converged, uint32_t flags);

int dg_tc_read(dg_query *q, uint64_t *count);

/* dg_pr_read for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments
 * and the same ranks, bit for bit, but no allocation of any kind.  Its partial
 * sums and the staging of a host copy use a fixed 4 MiB array in device memory,
 * one per GPU, held until the process ends.  With DG_DEVICE_PTRS any n is
 * accepted; a host rank buffer is staged through that array, so n above
 * DG_NOALLOC_MAX_HOST_N gives DG_EINVAL.  Calls share the array: the library
 * runs them one at a time per process (each returns after its copy is done);
 * other processes have their own copy. */
#define DG_NOALLOC_MAX_HOST_N 522240
int dg_pr_read_noalloc(dg_query *q, double *rank, int32_t *iters, int32_t *converged, uint32_t flags);

/* ---- checkpoint / resume of query state ---------------------------------------------- */

/* Serialise an attached query of a single graph (not of a set) into a host byte
 * buffer that dg_query_import accepts, also in another process, on a graph
 * re-created from dg_graph_export's edge list (the paper maintains these values
 * across batches, Section "StarPlat Dynamic: Programming Model"; saving them lets
 * that maintenance resume without a static recompute).  Contents, all in the
 * caller's vertex ids: a 64-byte header (kind, n, live edge count, parameters,
 * iteration count, triangle count) and then SSSP dist[n] and parent[n] (int32),
 * PageRank x[n] (double: the unnormalised values the Jacobi iteration keeps,
 * rank = x / sum(x)), or nothing for triangles.  Call with buf == NULL to get the
 * size in *bytes; otherwise *bytes holds the capacity on entry (DG_EINVAL if too
 * small) and receives the size written.  The caller owns buf. */
int dg_query_export(dg_query *q, void *buf, int64_t *bytes);

/* Attach a query to g from an exported buffer (host memory, read only during the
 * call), without the static solve.  DG_EINVAL, with nothing attached, when the
 * buffer is not an export, or its n or live edge count differ from g's, or:
 *   - SSSP: the distances and parents are not the shortest-path solution of g
 *     from the source (checked in one pass over g's arcs: no arc improves a
 *     distance, and every reachable vertex has a tight arc from its parent);
 *   - PageRank: a value is negative or not finite.  The values are a warm start:
 *     the Jacobi iteration runs until its L1 step meets the tolerance again (one
 *     step for a state exported from this edge set);
 *   - triangles: g is directed.  The count is taken as given, so it must come
 *     from an export of the same edge set.
 * On success *q is attached as by dg_*_attach. */
int dg_query_import(dg_graph *g, const void *buf, int64_t bytes, dg_query **q);

/* ---- batched sets of independent graphs ------------------------------------------------ */

/* Many independent directed graphs kept as one device-resident store and updated
 * together (the paper's Batch construct, Section 3.3.1, applied across graphs).
 * Member i has n[i] vertices and m[i] arcs; the arcs of all members are
 * concatenated in src/dst/w (w may be NULL: weight 1) with member-local vertex
 * ids.  flags may hold DG_DEVICE_PTRS for src/dst/w (n and m are host arrays).
 * Shortest-path updates run as frontier rounds with device-side counts, captured
 * once into hipGraphs and replayed for every batch (cfg->sssp_persistent 2, the
 * default for a set); cfg->sssp_persistent 1 asks for the persistent work queue
 * instead, also replayed from a captured hipGraph. */
typedef struct dg_set dg_set;
int dg_set_create(int32_t count, const int32_t *n, const int64_t *m, const int32_t *src,
                  const int32_t *dst, const int32_t *w, uint32_t flags, const dg_config *cfg,
                  dg_set **out);
int dg_set_destroy(dg_set *s);
/* Members, total vertices and total live arcs. */
int dg_set_info(dg_set *s, int32_t *count, int64_t *vertices, int64_t *arcs);
/* Attach shortest paths from member-local vertex sources[i] of every member
 * (static solve of every member; staticSSSP of Appendix A). */
int dg_set_sssp_attach(dg_set *s, const int32_t *sources);
/* Apply one update batch per member and bring every member's distances up to
 * date (DynSSSP of Appendix A).  k[i] updates for member i (host array),
 * concatenated in src/dst/w/op with member-local ids, semantics as
 * dg_apply_batch.  An id outside [0, n[i]) for its member, or any other invalid
 * update, rejects the whole call with DG_EINVAL before any change. */
int dg_set_apply_sssp(dg_set *s, const int64_t *k, const int32_t *src, const int32_t *dst,
                      const int32_t *w, const uint8_t *op, uint32_t flags, dg_batch_stats *stats);
/* Distances / parents of member i (member-local ids; n[i] entries each, parent
 * may be NULL).  Host pointers unless DG_DEVICE_PTRS. */
int dg_set_sssp_read(dg_set *s, int32_t member, int32_t *dist, int32_t *parent, uint32_t flags);
/* hipGraph replays and captures so far (a capture happens on the first batch and
 * whenever a buffer of the store is reallocated). */
int dg_set_graph_stats(dg_set *s, int64_t *launches, int64_t *captures);

/* ---- serving ------------------------------------------------------------------------- */

/* A request loop over resident graphs.  This is not in the paper; the Batch
 * construct of Section 3.3.1 is applied per request.  Every resident directed
 * graph keeps a PageRank (damping 0.85, L1 tolerance 1e-9) and a symmetrised
 * undirected copy with a triangle count: {u,v} is an edge of the copy while
 * (u,v) or (v,u) is an arc.
 *
 * A request is one update batch for one graph plus one query:
 *   - kind 0: distances from `source`, written to out (int32[n]);
 *   - kind 1: PageRank, written to out (double[n]);
 *   - kind 2: triangle count of the copy, also written to out (uint64, nullable).
 *
 * Scheduling.  `workers` threads each own a HIP stream.  A free worker takes the
 * oldest waiting request of a graph no other worker holds, once the request's
 * device-memory estimate fits under budget_bytes together with the running
 * requests.  So work for different graphs overlaps, and requests of one graph run
 * in arrival order, with results equal to running that sequence alone.
 *
 * Submission.  Submit copies the batch and returns at once:
 *   - DG_EBUSY when max_waiting requests already wait;
 *   - DG_EBUDGET when one request alone exceeds the budget.
 * The caller's out buffer must stay valid until the request is waited for.
 *
 * Clock.  Times are seconds since dg_server_start. */
typedef struct dg_server dg_server;
typedef struct dg_server_config {
    int32_t workers;       /* worker threads / streams; 0 = 4 */
    int32_t reserved0;
    int64_t budget_bytes;  /* device bytes for running requests; 0 = 8 GiB */
    int64_t max_waiting;   /* 0 = 2^20 */
} dg_server_config;
typedef struct dg_request {
    int32_t graph;
    int32_t kind;          /* 0 SSSP, 1 PageRank, 2 triangles */
    int32_t source;
    int32_t reserved0;
    int64_t k;             /* updates in the batch (may be 0) */
    const int32_t *src, *dst, *w; /* host arrays; w nullable (weight 1) */
    const uint8_t *op;     /* 0 delete, 1 insert */
    void *out;             /* host result buffer (see above) */
} dg_request;
typedef struct dg_result {
    int32_t status;        /* DG_OK or the error of the request */
    int32_t pr_iters;
    double t_submit, t_start, t_end;
    int64_t applied;       /* edges deleted + inserted in the directed graph */
    uint64_t tc;
    char error[96];        /* message of a failed request (status != DG_OK), else "" */
} dg_result;
int dg_server_create(const dg_server_config *cfg, dg_server **out);
/* Add a directed graph (host arrays; see dg_graph_create) before start. */
int dg_server_add_graph(dg_server *s, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                        const int32_t *w, const dg_config *cfg, int32_t *graph_id);
int dg_server_start(dg_server *s);
int dg_server_submit(dg_server *s, const dg_request *req, int64_t *ticket);
/* Block until the request ends (timeout < 0: no limit) and release its ticket;
 * DG_ENOTFOUND on timeout (the ticket stays valid) or for an unknown ticket. */
int dg_server_wait(dg_server *s, int64_t ticket, double timeout_s, dg_result *res);
/* Non-blocking form of dg_server_wait. */
int dg_server_poll(dg_server *s, int64_t ticket, dg_result *res);
/* Requests waiting for a worker, device bytes of the running ones. */
int dg_server_stats(dg_server *s, int64_t *waiting, int64_t *inflight_bytes);
/* Stop the workers after the running requests and free everything. */
int dg_server_destroy(dg_server *s);

/* ---- tuning ------------------------------------------------------------------------ */

/* Time candidate tile shapes (rows split above heavy_degree in {32..512},
 * persistent workgroups in {256..2048} where relevant) on one batch of updates
 * (same arguments as dg_apply_batch, applied to a device snapshot and rolled back
 * after every trial, so the graph is unchanged), keep the fastest in the graph's
 * configuration and report it in *best (nullable) with its time in *best_ms. */
int dg_autotune(dg_graph *g, int64_t k, const int32_t *src, const int32_t *dst, const int32_t *w,
                const uint8_t *op, uint32_t flags, dg_config *best, double *best_ms);
/* The same for a set, with one batch per member (arguments of dg_set_apply_sssp). */
int dg_set_autotune(dg_set *s, const int64_t *k, const int32_t *src, const int32_t *dst,
                    const int32_t *w, const uint8_t *op, uint32_t flags, dg_config *best,
                    double *best_ms);

/* ---- kernel timing ---------------------------------------------------------------- */

/* Per-kernel totals collected while profiling is on: launches, summed duration
 * (HIP events recorded on the stream each launch runs on) and summed algorithmic
 * bytes -- the bytes the method must move per launch, as documented per kernel
 * (not hardware counters). */
typedef struct dg_kernel_prof {
    char name[32];
    int64_t launches;
    double ms;
    double bytes;
} dg_kernel_prof;

/* Turn launch timing on (1) or off (0) for every graph of the process.  Timing
 * adds two event records per profiled launch and no synchronisation. */
int dg_profile_enable(int32_t on);
/* Drop all collected totals. */
int dg_profile_reset(void);
/* Wait for profiled work to finish and copy up to cap entries; *count gets the
 * number of kernels with totals. */
int dg_profile_read(dg_kernel_prof *out, int32_t cap, int32_t *count);

/* ---- sort and scan primitives (device memory) ---------------------------------------- */

/* The primitives the batch canonicalisation and the CSR maintenance are built on
 * (the sorted update batches that updateCSRDel / updateCSRAdd consume, Section
 * "Modified Graph Representation: diff-CSR"), exposed for callers and tests.
 * All pointers are device memory; work runs on `stream` (NULL: null stream) and
 * the call returns when it is done.  Calls are serialised within the process
 * (they share one workspace, allocated on first use and grown as needed).
 *
 * dg_sort_pairs: stable sort of n (key, value) pairs by the low `bits` bits of the
 * keys (1..64; higher bits are ignored for ordering but kept), least significant
 * digit first.  kin/vin are not modified; kout/vout receive the sorted pairs and
 * must not alias the inputs.  n < 2^31.
 *
 * dg_scan_exclusive: out[i] = in[0] + ... + in[i-1] for non-negative values whose
 * total stays below 2^48; out may equal in. */
int dg_sort_pairs(const uint64_t *kin, uint64_t *kout, const int32_t *vin, int32_t *vout, int64_t n, int32_t bits,
                  void *stream);
int dg_scan_exclusive(const int64_t *in, int64_t *out, int64_t n, void *stream);

/* ---- measurement ---------------------------------------------------------------------- */

/* Kernels with known memory traffic, for scaling hardware byte counters (the
 * roofline figures of the Experimental Evaluation comparisons rest on them):
 * kind 0 reads `bytes` bytes of device buffer `buf` once, kind 1 writes them once,
 * kind 2 reads one 4-byte word from each 128-byte line of them, kind 3 makes 2^26
 * 8-byte reads at pseudo-random positions (a SplitMix64 hash of the read index)
 * within them, the access pattern of a scattered gather over a working set of
 * `bytes` (the rate of the PageRank pull's contribution gathers depends on which
 * cache level holds that set).  bytes must be a multiple of 4 KiB (kind 3: at
 * least 64 KiB); the buffer's contents are overwritten (kinds 1, 2, and the first
 * 64 KiB for kind 3) or kept (kind 0).  Runs on `stream` (NULL: null stream) and
 * returns when done. */
int dg_calibrate(int32_t kind, void *buf, int64_t bytes, void *stream);

/* Floor under the whole-graph PageRank pull (the Jacobi sweep of the Appendix A
 * PR listings): a kernel that only streams the graph's base reverse columns (8
 * per lane, coalesced) and gathers one 8-byte value at each column, summed per
 * workgroup.  The pull does the same gathers plus the row sums and the stores, so
 * the ratio of the two times says how far the pull is from its gather bound.
 * Two warm-up launches, then `reps` (>= 1) timed ones with HIP events on the
 * graph's stream; *us = microseconds per launch.  Uses library scratch only. */
int dg_pr_gather_floor(dg_graph *g, int32_t reps, double *us);

/* ---- static recompute on the current graph (comparators) -------------------------- */

/* The "static" baseline of the paper's Experimental Evaluation section: the
 * updates are applied first and the property is then computed from scratch on
 * the updated graph (staticSSSP, staticPR and staticTC of Appendix A).  These
 * calls do the from-scratch part on the graph as it stands and leave attached
 * queries untouched.  dg_sssp_static: distances and parents from source, as
 * dg_sssp_read (flags: DG_DEVICE_PTRS).  dg_pr_static: Jacobi from 1/n to the L1
 * tolerance, ranks normalised as dg_pr_read, iterations in *iters (nullable).
 * dg_tc_static: undirected graphs only; merges the diff level first, then counts
 * each triangle once at its lowest-ranked vertex (forward algorithm). */

int dg_sssp_static(dg_graph *g, int32_t source, int32_t *dist, int32_t *parent, uint32_t flags);
int dg_pr_static(dg_graph *g, double damping, double tol, int32_t max_iter, double *rank,
                 int32_t *iters, uint32_t flags);
int dg_tc_static(dg_graph *g, uint64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
