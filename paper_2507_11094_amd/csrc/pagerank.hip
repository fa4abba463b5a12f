// PageRank: static Jacobi solve and the delta update on the affected set.
//
// The iteration is the one of the Appendix A PR listings (staticPR and the
// Incremental/Decremental steps): double-buffered Jacobi,
//     x'[v] = (1 - d)/n + d * sum_{u -> v} x[u] / outdeg(u),
// repeated while the L1 step exceeds the tolerance and the iteration cap is not
// reached, in FP64.  Like the listing, vertices without out-edges pass nothing
// on; the ranks the library returns are x / sum(x), which equals the usual
// PageRank with dangling mass spread uniformly (the fixed point of the
// dangling-dropped system, normalised, satisfies the dangling-uniform equation
// because the dangling redistribution vector equals the teleport vector).  Keeping
// the dangling-dropped system is what makes the update local.
//
// Delta update for one batch (DynPR: OnDelete/OnAdd flag the heads of changed
// arcs, propagateNodeFlags spreads the flags, Decremental/Incremental iterate on
// the flagged vertices):
//   seeds  = heads of every deleted or inserted arc, plus all current
//            out-neighbours of every tail (their share x[u]/outdeg(u) changed);
//   A      = everything reachable from the seeds along out-edges of the new graph
//            (the complement of A has no in-edge from A and no changed in-edge, so
//            its old values still satisfy the fixed-point equations);
//   Jacobi on A only, warm-started from the previous x, until the L1 step <= tol.
//
// Two iteration forms share the kernels (only the constant term differs):
//   local  (the listing's): x' = d P^T x + (1-d)/n, on A only.  Its error decays
//          like (d * rho)^k, rho the spectral radius of P^T on the recirculating
//          core (measured ~0.80 per step on R-MAT), hence many iterations.
//   global (dangling mass spread uniformly): y' = d P^T y + ((1-d) S + d D(y))/n
//          with S = sum(y) (conserved) and D(y) the mass on dangling vertices.  Its
//          fixed point is S * PageRank and it contracts at the second eigenvalue
//          of the Google matrix (~0.46 per step measured on R-MAT), but every
//          vertex moves each step.  Used for the static solve and for batches whose
//          affected set already covers most edges (auto: >= 20% of them), where
//          locality buys nothing; the result is rescaled to the local form's
//          fixed point, x = (1-d) / ((1-d) S + d D(y)) * y, so the next small batch
//          can continue locally.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "traverse.h"

namespace dg {

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

constexpr int APPLY_GROUPS = 1024;

__global__ void k_pr_init(int32_t n, double *x, double *contrib, const int32_t *deg) {
    const double x0 = 1.0 / (double)n;
    for (int64_t v = gtid(); v < n; v += gstride()) {
        x[v] = x0;
        contrib[v] = deg[v] > 0 ? x0 / (double)deg[v] : 0.0;
    }
}

// Pull for the vertices of A (A == nullptr: all vertices): xn[v] = base + d * sum
// of contrib over live in-edges.  Light vertices: a wave walks the edges of 64
// vertices 64 slots at a time and reduces each vertex's slots with a segmented
// scan in a fixed lane order; heavy vertices are cut into chunks (partial sums in
// `part`, combined in chunk order by k_pr_finish).  Deterministic throughout.
__global__ __launch_bounds__(256) void k_pr_pull(const int32_t *A, int64_t na, DirView g,
                                                 const double *__restrict__ contrib, const double *cterm,
                                                 double damp, double *xn, int64_t *hq, int64_t *hcount,
                                                 int64_t *hv, int64_t *hvcount, int heavy_deg, int chunk,
                                                 const double *done) {
    if (*done != 0.0) return;
    __shared__ double sacc[4][WAVE];
    const double base = *cterm;
    const int wslot = threadIdx.x / WAVE;
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    for (int64_t wb = wave_global * WAVE; wb < na; wb += nwaves * WAVE) {
        const int64_t fi = wb + l;
        int32_t v = -1;
        int64_t ob = 0, od = 0;
        int32_t db = 0, tot = 0;
        if (fi < na) {
            v = A ? A[fi] : (int32_t)fi;
            ob = g.off[v];
            db = (int32_t)(g.off[v + 1] - ob);
            od = g.doff[v];
            tot = db + (int32_t)(g.doff[v + 1] - od);
        }
        const bool heavy = tot > heavy_deg;
        int32_t nch = heavy ? (tot + chunk - 1) / chunk : 0;
        int64_t incl_ch = wave_incl_scan((int64_t)nch);
        int64_t tot_ch = __shfl(incl_ch, WAVE - 1, WAVE);
        int64_t base_ch = 0;
        if (l == 0 && tot_ch > 0) base_ch = atomicAdd((unsigned long long *)hcount, (unsigned long long)tot_ch);
        base_ch = __shfl(base_ch, 0, WAVE);
        const int64_t slot0 = base_ch + incl_ch - nch;
        for (int32_t c = 0; c < nch; ++c) hq[slot0 + c] = ((int64_t)v << 32) | (uint32_t)c;
        int64_t hs = wave_append(hvcount, heavy);
        if (heavy) {
            hv[2 * hs] = ((int64_t)v << 32) | (uint32_t)nch;
            hv[2 * hs + 1] = slot0;
            tot = 0;
        }
        sacc[wslot][l] = 0.0;
        __builtin_amdgcn_wave_barrier();
        const int64_t incl = wave_incl_scan((int64_t)tot);
        const int64_t excl = incl - tot;
        const int64_t T = __shfl(incl, WAVE - 1, WAVE);
        for (int64_t eb = 0; eb < T; eb += WAVE) {
            const int64_t e = eb + l;
            int o = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                int cand = o + step;
                int64_t x = __shfl(excl, cand, WAVE);
                if (x <= e) o = cand;
            }
            const int64_t obo = __shfl(ob, o, WAVE);
            const int64_t odo = __shfl(od, o, WAVE);
            const int32_t dbo = __shfl(db, o, WAVE);
            const int64_t exo = __shfl(excl, o, WAVE);
            double val = 0.0;
            if (e < T) {
                int64_t j = e - exo;
                uint32_t c = j < dbo ? (uint32_t)g.col[obo + j] : (uint32_t)g.dcol[odo + (j - dbo)];
                if (!(c & DEAD)) val = contrib[c & ID_MASK];
            }
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                double y = __shfl_up(val, d, WAVE);
                int oo = __shfl_up(o, d, WAVE);
                if (l >= d && oo == o) val += y;
            }
            int on = __shfl_down(o, 1, WAVE);
            if (l == WAVE - 1 || on != o) sacc[wslot][o] += val;
            __builtin_amdgcn_wave_barrier();
        }
        if (v >= 0 && !heavy) xn[v] = base + damp * sacc[wslot][l];
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ __launch_bounds__(256) void k_pr_heavy(DirView g, const double *__restrict__ contrib,
                                                  const int64_t *hq, const int64_t *hcount, int chunk,
                                                  double *part) {
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    const int64_t nq = *hcount;
    for (int64_t qi = wave_global; qi < nq; qi += nwaves) {
        const int64_t ent = hq[qi];
        const int32_t v = (int32_t)(ent >> 32);
        const int32_t c = (int32_t)(ent & 0xffffffff);
        const int64_t ob = g.off[v];
        const int32_t db = (int32_t)(g.off[v + 1] - ob);
        const int64_t od = g.doff[v];
        const int32_t tot = db + (int32_t)(g.doff[v + 1] - od);
        const int64_t s = (int64_t)c * chunk;
        const int64_t e = min((int64_t)tot, s + chunk);
        double acc = 0.0;
        for (int64_t j = s + l; j < e; j += WAVE) {
            uint32_t cc = j < db ? (uint32_t)g.col[ob + j] : (uint32_t)g.dcol[od + (j - db)];
            if (!(cc & DEAD)) acc += contrib[cc & ID_MASK];
        }
        acc = wave_sum(acc);
        if (l == 0) part[qi] = acc;
    }
}

__global__ void k_pr_finish(const int64_t *hv, const int64_t *hvcount, const double *part,
                            const double *cterm, double damp, double *xn) {
    const int64_t nh = *hvcount;
    const double base = *cterm;
    for (int64_t i = gtid(); i < nh; i += gstride()) {
        const int32_t v = (int32_t)(hv[2 * i] >> 32);
        const int32_t nch = (int32_t)(hv[2 * i] & 0xffffffff);
        const int64_t s0 = hv[2 * i + 1];
        double sum = 0.0;
        for (int32_t c = 0; c < nch; ++c) sum += part[s0 + c];
        xn[v] = base + damp * sum;
    }
}

// Fixed-order block reduction of two values.
__device__ __forceinline__ void block_sum2(double a, double b, double *out_a, double *out_b) {
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out_a = ra[0];
        *out_b = rb[0];
    }
}

// Fixed-order block sums of K more values (after block_sum2 in the same kernel).
template <int K>
__device__ __forceinline__ void block_sum_more(const double (&v)[K], double *out) {
    __shared__ double r[K][256];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) r[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < K; ++k) r[k][threadIdx.x] += r[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = r[k][0];
    }
}

// prs[0] = L1 step, prs[1] = dangling mass, prs[2] = constant term of the next
// step (global form: ((1-d) S + d D) / n; local form: (1-d) / n), prs[3] = 1 once
// the step is <= tol (every later kernel of the iteration then returns at once),
// prs[4] = steps taken, prs[5] = the step (copied for the host), prs[6] = |previous
// step|^2 (0: none comparable), prs[7] = the previous aligned ratio (0: none),
// prs[8] = the extrapolation factor the next apply uses (0: plain step),
// prs[9] = plain steps since the last move, prs[10] = moves taken, prs[11] = 1
// while the applies keep the step vector for the fits (stops after EX_TRACK plain
// steps without a move: error spread over many modes of different ratios never
// lines up, and the extra vector traffic would be paid on every step),
// prs[12] = |step before the previous|^2 (0: none comparable), prs[13] = the
// conserved mass (S < 0), prs[14] = 1 when the move of the next apply is a
// two-step move, prs[15] = 1 once the applies also keep the step before the
// previous one (after EX_LAG2_AFTER plain steps without a move, on a step whose
// one-step fit left at least EX_LAG2_RES of |s_k|^2 unexplained: on a grid the
// successive steps are orthogonal, while on R-MAT graphs from scale 16 up the fit
// explains more than 20 % by the fourth step in the CPU models and the older
// vector is not kept; where it is, on small graphs, no two-step move fired).
// first = 1: the set-up call before the first step (resets the flags and counts).
//
// Extrapolation (extrap = 1, partials2 holds the block sums of |step|^2,
// <step, previous step> and <step, step before the previous>): the step vectors of
// a linear fixed-point iteration shrink like e_{k+1} = M e_k.  When the error is
// dominated by one eigenvector of M with eigenvalue lam, successive steps are
// parallel, s_k = lam s_{k-1}, and x + lam / (1 - lam) (x' - x) removes that
// component (Aitken's delta-squared process along the step).  lam is fitted by
// least squares, lam = <s_k, s_{k-1}> / |s_{k-1}|^2, and the move is taken only
// when the fit leaves at most EX_FIT of |s_k| unexplained and
// 0 < lam <= EX_MAX_LAM.  (Asking for two successive aligned fits with ratios
// within 5 % as well delayed the move by one step and changed nothing else in the
// CPU models.)
// Bipartite graphs such as grids have their eigenvalues in pairs +-lam, so the
// error of a batch sits in modes near +d and -d at once and successive steps never
// line up.  Over two steps both modes of a pair shrink by mu = lam^2, so the fit
// of s_k against s_{k-2} (mu = <s_k, s_{k-2}> / |s_{k-2}|^2, at most EX_FIT2
// unexplained, 0 < mu <= EX_MAX_LAM^2) finds them, and the two-step map's Aitken
// move x + mu / (1 - mu) (x'' - x) goes along the sum of the last two steps.  This
// fit is only tried when the one-step fit is not taken.
// The next apply takes the move; a step that moved is never taken as converged,
// and the fits restart after it.  Convergence is only declared on a plain step,
// whose L1 size bounds the error exactly as in plain Jacobi, and a one-step move
// keeps sum(x) (an affine combination of two vectors of equal sum; the two-step
// move adds the previous step in FP32, a change of sum far below the tolerance).
constexpr double EX_FIT = 0.05;     // unexplained fraction of |s_k| (L2) at most
constexpr double EX_FIT2 = 0.15;    // the same for the fit against s_{k-2}
constexpr double EX_MAX_LAM = 0.9;  // no move for slower ratios (factor <= 9)
constexpr int EX_TRACK = 24;        // plain steps without a move before the fits stop
constexpr int EX_LAG2_AFTER = 4;    // plain steps without a move before s_{k-2} is kept,
constexpr double EX_LAG2_RES = 0.95;  // and the one-step fit explaining at most 5 % of |s_k|^2
__device__ __forceinline__ void pr_reduce_body(const double *partials, const double *partials2, int np, int global,
                                               double S, double damp, double ninv, double tol, int first, int extrap,
                                               double *prs, double *step_out) {
    double a = 0.0, b = 0.0, sq = 0.0, dot = 0.0, dot2 = 0.0;
    const bool fit = extrap && !first && prs[11] != 0.0;  // the apply just run kept the step vector
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
        if (fit) {
            sq += partials2[3 * i];
            dot += partials2[3 * i + 1];
            dot2 += partials2[3 * i + 2];
        }
    }
    __shared__ double fs[3];
    block_sum2(a, b, &prs[0], &prs[1]);
    if (fit) {
        const double v[3] = {sq, dot, dot2};
        block_sum_more<3>(v, fs);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // S < 0: the conserved mass is prs[13], set by the set-up call (first) to the
        // sum of the start vector (prs[0] then), and tol is relative to it
        if (first && S < 0.0) prs[13] = prs[0];
        if (S < 0.0) {
            S = prs[13];
            tol *= prs[13];
        }
        prs[2] = global ? ((1.0 - damp) * S + damp * prs[1]) * ninv : (1.0 - damp) * ninv;
        *step_out = prs[0];
        if (first) {
            prs[3] = 0.0;
            prs[4] = 0.0;
            for (int k = 6; k <= 10; ++k) prs[k] = 0.0;
            prs[11] = extrap ? 1.0 : 0.0;
            prs[12] = 0.0;
            prs[14] = 0.0;
            prs[15] = 0.0;
            return;
        }
        prs[4] += 1.0;
        const double step = prs[0];
        const bool moved = prs[8] != 0.0;
        prs[8] = 0.0;
        prs[14] = 0.0;
        if (moved) {
            // the step just taken moved further than Jacobi: the fits start again
            prs[6] = 0.0;
            prs[7] = 0.0;
            prs[9] = 0.0;
            prs[12] = 0.0;
            prs[11] = extrap ? 1.0 : 0.0;
            return;
        }
        if (step <= tol) {
            prs[3] = 1.0;
            return;
        }
        if (!fit) return;
        prs[9] += 1.0;
        const bool lag2 = prs[15] != 0.0;  // the apply just run kept s_{k-2} as well
        const double s2 = fs[0], sd = fs[1], sd2 = fs[2], p2 = prs[6], q2 = prs[12];
        const double lam = p2 > 0.0 ? sd / p2 : 0.0;
        const bool aligned = p2 > 0.0 && s2 - sd * lam <= EX_FIT * EX_FIT * s2;
        const double mu = q2 > 0.0 ? sd2 / q2 : 0.0;
        const bool aligned2 = q2 > 0.0 && s2 - sd2 * mu <= EX_FIT2 * EX_FIT2 * s2;
        if (aligned && lam > 0.0 && lam <= EX_MAX_LAM && prs[9] >= 2.0 && lam * step > 2.0 * tol) {
            prs[8] = lam / (1.0 - lam);
            prs[10] += 1.0;
        } else if (aligned2 && mu > 0.0 && mu <= EX_MAX_LAM * EX_MAX_LAM && mu * step > 2.0 * tol) {
            prs[8] = mu / (1.0 - mu);
            prs[14] = 1.0;
            prs[10] += 1.0;
        }
        prs[7] = aligned ? lam : 0.0;
        prs[12] = lag2 ? p2 : 0.0;  // the apply just run stored s_{k-1} as the older vector
        prs[6] = s2;
        if (prs[9] >= (double)EX_LAG2_AFTER && p2 > 0.0 && s2 - sd * lam >= EX_LAG2_RES * s2) prs[15] = 1.0;
        // a two-step move needs the step vector in the next apply: tracking stops
        // only on a step that decided no move, after EX_TRACK plain steps or once
        // the step is too small for any move (the move tests above fail for it)
        if (prs[8] == 0.0 && (prs[9] >= (double)EX_TRACK || EX_MAX_LAM * EX_MAX_LAM * step <= 2.0 * tol))
            prs[11] = 0.0;
    }
}

__global__ void k_pr_reduce(const double *partials, const double *partials2, int np, int global, double S,
                            double damp, double ninv, double tol, int first, int extrap, double *prs,
                            double *step_out) {
    if (!first && prs[3] != 0.0) return;
    pr_reduce_body(partials, partials2, np, global, S, damp, ninv, tol, first, extrap, prs, step_out);
}

// contrib := xn / outdeg on A, and x := xn unless x_w is null (the whole-graph
// steps alternate two buffers instead of copying); fixed-order partials of the L1
// step |xn - x_o| and of the new mass on dangling vertices (k_pr_reduce sums
// them).  Summing them in the last workgroup to finish instead (an atomic ticket
// after a device-scope fence per workgroup) took 62-68 us per step against 22 + 4
// us for the two launches: the fence writes the L2 back in every workgroup.
__global__ __launch_bounds__(256) void k_pr_apply(const int32_t *A, int64_t na, double *xn,
                                                  const double *x_o, double *x_w, double *contrib,
                                                  const int32_t *deg, double *partials, double *partials2,
                                                  float *dprev, float *dprev2, const double *prs) {
    if (prs[3] != 0.0) return;
    // dprev (extrapolation on) while prs[11] != 0: the previous step's vector is read
    // and this step's written (FP32: it only feeds the fits), and partials2 gets the
    // block sums of |step|^2, <step, previous step> and <step, step before it>.
    // dprev2 while prs[15] != 0 as well: the step before the previous one is read and
    // the previous one moves into its place.  f = prs[8] != 0: the new vector also
    // moves f times this step further, or f times the sum of this step and the
    // previous one (prs[14] != 0, a two-step move); the L1 step summed is the plain one.
    const double f = prs[8];
    const bool two = prs[14] != 0.0;
    if (dprev && prs[11] == 0.0) dprev = nullptr;
    if (!dprev || prs[15] == 0.0) dprev2 = nullptr;
    double acc = 0.0, dang = 0.0, sq = 0.0, dot = 0.0, dot2 = 0.0;
    // four strided elements per pass, every load issued before the stores (x_w may be
    // x_o, so the compiler could not reorder them itself); the sums keep the order
    // of a plain strided loop
    constexpr int U = 4;
    const int64_t st = gstride();
    for (int64_t i0 = gtid(); i0 < na; i0 += U * st) {
        int32_t v[U], dg[U];
        double nv[U], ov[U], pv[U], pv2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * st;
            v[u] = i < na ? (A ? A[i] : (int32_t)i) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v[u] < 0) continue;
            nv[u] = xn[v[u]];
            ov[u] = x_o[v[u]];
            dg[u] = deg[v[u]];
            pv[u] = dprev ? (double)dprev[v[u]] : 0.0;
            pv2[u] = dprev2 ? (double)dprev2[v[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v[u] < 0) continue;
            const double dl = nv[u] - ov[u];
            acc += fabs(dl);
            if (dprev) {
                sq += dl * dl;
                dot += dl * pv[u];
                if (dprev2) {
                    dot2 += dl * pv2[u];
                    dprev2[v[u]] = (float)pv[u];
                }
                dprev[v[u]] = (float)dl;
            }
            double y = nv[u];
            if (f != 0.0) {
                y = nv[u] + f * (two ? dl + pv[u] : dl);
                if (!x_w) xn[v[u]] = y;
            }
            if (x_w) x_w[v[u]] = y;
            contrib[v[u]] = dg[u] > 0 ? y / (double)dg[u] : 0.0;
            if (dg[u] == 0) dang += y;
        }
    }
    block_sum2(acc, dang, &partials[2 * blockIdx.x], &partials[2 * blockIdx.x + 1]);
    if (dprev2) {
        const double v3[3] = {sq, dot, dot2};
        block_sum_more<3>(v3, &partials2[3 * blockIdx.x]);
    } else if (dprev) {
        const double v2[2] = {sq, dot};
        block_sum_more<2>(v2, &partials2[3 * blockIdx.x]);
        if (threadIdx.x == 0) partials2[3 * blockIdx.x + 2] = 0.0;
    }
}

// Sum and dangling mass of a whole vector: partials for k_pr_reduce.
__global__ __launch_bounds__(256) void k_sum_vec2(const double *x, const int32_t *deg, int64_t n,
                                                  double *partials) {
    double a = 0.0, b = 0.0;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        a += x[i];
        if (deg[i] == 0) b += x[i];
    }
    block_sum2(a, b, &partials[2 * blockIdx.x], &partials[2 * blockIdx.x + 1]);
}

// Scale a global-form solution y to the local form's fixed point:
// x = (1-d) / ((1-d) S + d D(y)) * y, contrib = x / outdeg.
__global__ void k_pr_rescale(int32_t n, double *x, double *contrib, const int32_t *deg, const double *prs,
                             double S, double damp) {
    if (S < 0.0) S = prs[13];  // the mass kept on the device
    const double alpha = (1.0 - damp) / ((1.0 - damp) * S + damp * prs[1]);
    for (int64_t v = gtid(); v < n; v += gstride()) {
        double nv = x[v] * alpha;
        x[v] = nv;
        int32_t dg = deg[v];
        contrib[v] = dg > 0 ? nv / (double)dg : 0.0;
    }
}

__global__ void k_sum_partials(const double *partials, int np, double *out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ __launch_bounds__(256) void k_sum_vec(const double *x, int64_t n, double *partials) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = gtid(); i < n; i += gstride()) acc += x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// out[i] = x[perm[i]] / sum: ranks in the caller's ids (perm null: ids kept).
__global__ void k_scale(const double *x, const int32_t *perm, int64_t n, const double *sum, double *out) {
    const double s = *sum;
    for (int64_t i = gtid(); i < n; i += gstride()) out[i] = x[perm ? perm[i] : i] / s;
}

// Reach closure and seeds.
struct ReachOp {
    int32_t *stamp;
    int32_t st;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t, int32_t &pay) const { pay = 0; return true; }
    __device__ bool edge(bool valid, int32_t, int32_t, int32_t x, int32_t) const {
        // plain load first: most edges reach vertices that are already marked
        return valid && stamp[x] != st && atomicExch(&stamp[x], st) != st;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

// Mark a list of vertices with stamp st; append the first-time ones to out.
__global__ void k_mark_list(int64_t n, const int32_t *a, int32_t *stamp, int32_t st, int32_t *out,
                            int64_t *count) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += gstride()) {
        int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < n) {
            v = a[i];
            p = atomicExch(&stamp[v], st) != st;
        }
        int64_t slot = block_append(count, p, sc);
        if (p) out[slot] = v;
    }
}

// Affected set in vertex order (deterministic sums and near-contiguous row reads).
__global__ void k_stamp_flags(int32_t n, const int32_t *stamp, int32_t st, int64_t *flags) {
    for (int64_t v = gtid(); v <= n; v += gstride()) flags[v] = v < n && stamp[v] == st;
}
__global__ void k_compact_flags(int32_t n, const int64_t *flags, const int64_t *pos, int32_t *out) {
    for (int64_t v = gtid(); v < n; v += gstride())
        if (flags[v]) out[pos[v]] = (int32_t)v;
}

__global__ void k_refresh_contrib(const int64_t *n_p, const int32_t *u, const double *x, const int32_t *deg,
                                  double *contrib) {
    const int64_t n = *n_p;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        int32_t v = u[i];
        int32_t dg = deg[v];
        contrib[v] = dg > 0 ? x[v] / (double)dg : 0.0;
    }
}

// ---- host side ---------------------------------------------------------------------------

static int heavy_deg(dg_graph *g) { return g->cfg.heavy_degree > 0 ? g->cfg.heavy_degree : 512; }

// ---- whole-graph pull: merge-path tiles ---------------------------------------------
// When every vertex is pulled (static solve, global form) the pull is a sparse
// matrix-vector product over the reverse CSR.  The row ends and the base entries
// form one merged sequence of n + m items; tile b takes the items
// [b * MP_ITEMS, (b + 1) * MP_ITEMS) of it (the merge-path decomposition of
// Merrill and Garland, PPoPP 2016), so every workgroup streams the same amount of
// work whatever the degree skew: no per-vertex wave, no heavy-row queue.
//   k_mp_partition  tile start coordinates (row, entry), once per iteration call;
//   k_pr_tiles      entries staged through LDS (column reads coalesced, one
//                   contribution gather per entry), then each row that ends in
//                   the tile is summed in entry order: short pieces by one lane,
//                   long pieces by a wave; rows that began in an earlier tile
//                   leave their piece in pf[b], the row still open at the tile's
//                   end leaves its piece in pl[b];
//   k_pr_rows       rows split across tiles: pieces added in tile order, then
//                   their diff-level entries; the other rows' diff-level entries
//                   added per row in key order.
// Every sum has a fixed order, so results are bit-reproducible.
constexpr int MP_THREADS = 256;
constexpr int MP_ITEMS = 2048;  // default items per tile (cfg.pr_tile picks 1024 / 2048 / 4096)
constexpr int MP_LONG = 64;     // row pieces longer than this are summed by a whole wave

__global__ void k_mp_partition(const int64_t *__restrict__ off, int32_t n, int64_t m, int64_t nb, int items,
                               int32_t *mp_row, int64_t *mp_edge) {
    for (int64_t b = gtid(); b <= nb; b += gstride()) {
        const int64_t diag = min(b * (int64_t)items, (int64_t)n + m);
        // rows consumed at this diagonal: the largest r with off[r] <= diag - r
        // (a row's end is taken before the entry that starts the next row)
        int64_t lo = max(diag - m, (int64_t)0), hi = min(diag, (int64_t)n);
        while (lo < hi) {
            const int64_t p = (lo + hi) >> 1;
            if (off[p + 1] <= diag - p - 1) lo = p + 1;
            else hi = p;
        }
        mp_row[b] = (int32_t)lo;
        mp_edge[b] = diag - lo;
    }
}

// STREAM: the column and offset streams are read, and the results written, with
// non-temporal hints, so that they do not displace the gathered contributions
// from L2.
template <bool STREAM>
__device__ __forceinline__ int32_t ld_stream(const int32_t *p) {
    return STREAM ? __builtin_nontemporal_load(p) : *p;
}
template <bool STREAM>
__device__ __forceinline__ int64_t ld_stream(const int64_t *p) {
    return STREAM ? __builtin_nontemporal_load(p) : *p;
}
template <bool STREAM>
__device__ __forceinline__ void st_stream(double *p, double v) {
    if (STREAM) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <bool STREAM, int ITEMS>
__global__ __launch_bounds__(MP_THREADS) void k_pr_tiles(const int32_t *__restrict__ mp_row,
                                                         const int64_t *__restrict__ mp_edge,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ contrib, const double *cterm,
                                                         double damp, double *xn, double *pf, double *pl,
                                                         const double *done) {
    if (*done != 0.0) return;
    constexpr int IPT = ITEMS / MP_THREADS;
    __shared__ double s_val[ITEMS];
    __shared__ int32_t s_off[ITEMS + 1];
    __shared__ int32_t s_long[ITEMS / MP_LONG + 2];
    __shared__ int32_t s_nlong;
    const int64_t b = blockIdx.x;
    const int32_t r0 = mp_row[b], r1 = mp_row[b + 1];
    const int64_t e0 = mp_edge[b];
    const int32_t ne = (int32_t)(mp_edge[b + 1] - e0);
    const int32_t nr = r1 - r0;
    const int t = threadIdx.x;
    if (t == 0) s_nlong = 0;
    // stage the entries: all column loads first, the row starts while they are in
    // flight, then all gathers (IPT in flight per lane)
    uint32_t c[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int j = t + u * MP_THREADS;
        c[u] = j < ne ? (uint32_t)ld_stream<STREAM>(&col[e0 + j]) : DEAD;
    }
    // row starts relative to the tile (-1: the row began in an earlier tile)
    for (int i = t; i <= nr; i += MP_THREADS) {
        const int64_t o = ld_stream<STREAM>(&off[r0 + i]) - e0;
        s_off[i] = (int32_t)(o < 0 ? -1 : o);
    }
    double v[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) v[u] = (c[u] & DEAD) ? 0.0 : contrib[c[u] & ID_MASK];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int j = t + u * MP_THREADS;
        if (j < ne) s_val[j] = v[u];
    }
    __syncthreads();
    const double base = *cterm;
    // rows that end in this tile: short pieces one lane each
    for (int i = t; i < nr; i += MP_THREADS) {
        const int32_t lo = max(s_off[i], 0), hi = s_off[i + 1];
        if (hi - lo > MP_LONG) {
            s_long[atomicAdd(&s_nlong, 1)] = i;
            continue;
        }
        double acc = 0.0;
        for (int32_t j = lo; j < hi; ++j) acc += s_val[j];
        if (s_off[i] < 0) pf[b] = acc;
        else st_stream<STREAM>(&xn[r0 + i], base + damp * acc);
    }
    __syncthreads();
    // long pieces, then the piece of the row left open at the tile's end, one wave each
    const int wv = t / WAVE, l = lane_id();
    const int nlong = s_nlong;
    for (int k = wv; k <= nlong; k += MP_THREADS / WAVE) {
        int32_t lo, hi;
        if (k < nlong) {
            lo = max(s_off[s_long[k]], 0);
            hi = s_off[s_long[k] + 1];
        } else {
            lo = max(s_off[nr], 0);
            hi = ne;
        }
        double acc = 0.0;
        for (int32_t j = lo + l; j < hi; j += WAVE) acc += s_val[j];
        acc = wave_sum(acc);
        if (l == 0) {
            if (k == nlong) pl[b] = acc;
            else if (s_off[s_long[k]] < 0) pf[b] = acc;
            else st_stream<STREAM>(&xn[r0 + s_long[k]], base + damp * acc);
        }
    }
}

// After the tiles, one pass finishes two kinds of rows:
//   k < nb:  rows that began in an earlier tile and end in tile k: the open pieces
//            of the tiles before (pl, in tile order) plus the closing piece
//            (pf[k]), then the row's diff-level entries;
//   k >= nb: diff-level entries, the first entry of each row's run adding the
//            run's live contributions in key order -- except for rows split
//            across tiles, which the first kind finishes whole.
// A row r is split when its first entry and its end fall in different tiles of the
// merged sequence: items r + off[r] and r + off[r + 1] (a row's end comes after
// its entries and before the next row's first entry).
__global__ void k_pr_rows(int64_t nb, int items, const int32_t *__restrict__ mp_row,
                          const int64_t *__restrict__ mp_edge, const int64_t *__restrict__ off, const double *pf,
                          const double *pl, int64_t dm, const uint64_t *__restrict__ dkey,
                          const int64_t *__restrict__ doff, const int32_t *__restrict__ dcol, int keybits,
                          const double *__restrict__ contrib, const double *cterm, double damp, double *xn,
                          const double *done) {
    if (*done != 0.0) return;
    const double base = *cterm;
    for (int64_t k = gtid(); k < nb + dm; k += gstride()) {
        if (k < nb) {
            const int32_t R = mp_row[k];
            if (R >= mp_row[k + 1] || off[R] >= mp_edge[k]) continue;
            int64_t first = k - 1;  // tile k-1 ends inside row R
            while (first > 0 && mp_row[first] == R) --first;
            double acc = 0.0;
            for (int64_t j = first; j < k; ++j) acc += pl[j];
            acc += pf[k];
            double x = base + damp * acc;
            double dacc = 0.0;
            for (int64_t q = doff[R]; q < doff[R + 1]; ++q) {
                const uint32_t cc = (uint32_t)dcol[q];
                if (!(cc & DEAD)) dacc += contrib[cc & ID_MASK];
            }
            if (dacc != 0.0) x += damp * dacc;
            xn[R] = x;
        } else {
            const int64_t j = k - nb;
            const int32_t r = (int32_t)(dkey[j] >> keybits);
            if (j > 0 && (int32_t)(dkey[j - 1] >> keybits) == r) continue;
            if (((int64_t)r + off[r]) / items != ((int64_t)r + off[r + 1]) / items) continue;
            double acc = 0.0;
            for (int64_t q = j; q < dm && (int32_t)(dkey[q] >> keybits) == r; ++q) {
                const uint32_t cc = (uint32_t)dcol[q];
                if (!(cc & DEAD)) acc += contrib[cc & ID_MASK];
            }
            if (acc != 0.0) xn[r] += damp * acc;
        }
    }
}

// ---- gather floor --------------------------------------------------------------------
// The whole-graph pull gathers one 8-byte contribution per base entry at a scattered
// column.  This kernel does only that: the column stream (coalesced, 8 entries per
// lane as in the tiles) and the gathers, summed per workgroup, one write per
// workgroup.  Its time is the floor under k_pr_tiles for the same column order.
__global__ __launch_bounds__(256) void k_gather_floor(const int32_t *__restrict__ col, int64_t m,
                                                      const double *__restrict__ vals, double *out) {
    constexpr int LANE_ITEMS = 8;
    const int64_t e0 = (int64_t)blockIdx.x * 256 * LANE_ITEMS;
    uint32_t c[LANE_ITEMS];
#pragma unroll
    for (int u = 0; u < LANE_ITEMS; ++u) {
        const int64_t j = e0 + threadIdx.x + u * 256;
        c[u] = j < m ? (uint32_t)__builtin_nontemporal_load(&col[j]) : DEAD;
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < LANE_ITEMS; ++u) acc += (c[u] & DEAD) ? 0.0 : vals[c[u] & ID_MASK];
    acc = wave_sum(acc);
    __shared__ double part[256 / WAVE];
    if (lane_id() == 0) part[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / WAVE; ++w) t += part[w];
        out[blockIdx.x] = t;
    }
}

int pr_gather_floor(dg_graph *g, int32_t reps, double *us) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const Dir &R = *g->rev;
    const int64_t m = R.m;
    const int64_t blocks = (m + 2047) / 2048;
    DG_TRY(ws.rbuf.ensure((size_t)g->n + 1));
    DG_TRY(ws.sx.ensure((size_t)std::max<int64_t>(blocks, 1)));
    DG_HIP(hipMemsetAsync(ws.rbuf.p, 0, ((size_t)g->n + 1) * sizeof(double), s));
    *us = 0.0;
    if (m == 0 || reps <= 0) return DG_OK;
    hipEvent_t e0, e1;
    DG_HIP(hipEventCreate(&e0));
    DG_HIP(hipEventCreate(&e1));
    int rc = DG_OK;
    for (int i = 0; i < 2 + reps; ++i) {
        if (i == 2 && hipEventRecord(e0, s) != hipSuccess) rc = DG_EDEVICE;
        hipLaunchKernelGGL(k_gather_floor, dim3((unsigned)blocks), dim3(256), 0, s, R.col.p, m, ws.rbuf.p, ws.sx.p);
    }
    if (rc == DG_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess))
        rc = DG_EDEVICE;
    float ms = 0.0f;
    if (rc == DG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DG_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DG_OK) return set_error(rc, "gather floor: device error");
    *us = 1000.0 * (double)ms / (double)reps;
    return DG_OK;
}

static int ensure_pr_ws(dg_graph *g) {
    Work &ws = g->ws;
    DG_TRY(ws.f0.ensure((size_t)g->n + 1));
    DG_TRY(ws.f1.ensure((size_t)g->n + 1));
    int64_t edges = std::max(g->fwd.m + g->fwd.dm, g->rev->m + g->rev->dm);
    const int64_t qcap = 2 * (edges / heavy_deg(g) + 2) + g->n / 8 + 64;
    DG_TRY(ws.heavy.ensure((size_t)qcap * 2 + 2 * (size_t)qcap * 2));
    DG_TRY(ws.part.ensure((size_t)qcap + 5 * APPLY_GROUPS + 8));
    DG_TRY(ws.prs.ensure(16));
    return DG_OK;
}

// Total entries (base + diff, tombstones included) of the rows of A.
__global__ void k_sum_degrees(const int32_t *A, int64_t na, const int64_t *na_p, const int64_t *off,
                              const int64_t *doff, int64_t *out) {
    if (na_p) na = *na_p;
    int64_t acc = 0;
    for (int64_t i = gtid(); i < na; i += gstride()) {
        int32_t v = A[i];
        acc += (off[v + 1] - off[v]) + (doff[v + 1] - doff[v]);
    }
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd((unsigned long long *)out, (unsigned long long)acc);
}

// Jacobi on A (nullptr = all n vertices) until the L1 step <= tol or max_iter.
// global: the dangling-uniform form with conserved mass S (see the file header);
// otherwise the local form.  S < 0: the mass is the sum of x at the start, kept on
// the device, and tol is relative to it (no host round trip for it).  `edges` = entries scanned per pull (for the
// algorithmic byte count):
//   pull:  A[i] 4 + off 8 + doff 8 + xn write 8 per vertex, col 4 + contrib 8 per entry
//   apply: A[i] 4 + xn 8 + x read 8 + x write 8 + contrib write 8 + outdeg 4 per vertex;
//          whole-graph tiles: xn 8 + x read 8 + contrib write 8 + outdeg 4 (no A, and
//          the two vectors trade places instead of a copy)
static int pr_iterate(dg_graph *g, const int32_t *A, int64_t na, int64_t edges, double damping,
                      double tol, int32_t max_iter, bool global, double S, double *x, double *xn,
                      double *contrib, int32_t *iters, int32_t *conv, SideWork *side = nullptr,
                      int32_t first_group = 0) {
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int64_t qcap = 2 * (std::max(g->fwd.m + g->fwd.dm, g->rev->m + g->rev->dm) / heavy_deg(g) + 2) +
                         g->n / 8 + 64;
    int64_t *hq = reinterpret_cast<int64_t *>(ws.heavy.p);
    int64_t *hv = hq + qcap;
    double *partials = ws.part.p + qcap;
    const double ninv = 1.0 / (double)g->n;
    DirView rv = view(*g->rev);
    double *prs = ws.prs.p;
    double *const x_home = x, *const xn_home = xn;
    double *step_out = prs + 5;  // not in the shared counters: SSSP may run beside these steps
    ws.pr_moves = 0;
    // constant term of the first step (and, S < 0, the mass of the start vector)
    if (global || S < 0.0)
        hipLaunchKernelGGL(k_sum_vec2, dim3(APPLY_GROUPS), dim3(256), 0, s, x, g->fwd.deg.p, (int64_t)g->n,
                           partials);
    else
        hipLaunchKernelGGL(k_sum_vec2, dim3(1), dim3(256), 0, s, x, g->fwd.deg.p, (int64_t)0, partials);
    // extrapolated steps keep the last two step vectors (n floats each) and three
    // more sums per apply
    const int extrap = g->cfg.pr_extrapolate ? 1 : 0;
    double *partials2 = partials + 2 * APPLY_GROUPS;
    float *dprev = nullptr, *dprev2 = nullptr;
    if (extrap) {
        DG_TRY(ws.prstep.ensure((size_t)g->n + 1));
        DG_TRY(ws.prstep2.ensure((size_t)g->n + 1));
        dprev = ws.prstep.p;
        dprev2 = ws.prstep2.p;
    }
    hipLaunchKernelGGL(k_pr_reduce, dim3(1), dim3(256), 0, s, partials, partials2,
                       global || S < 0.0 ? APPLY_GROUPS : 1, (int)global, S, damping, ninv, tol, 1, extrap, prs,
                       step_out);
    DG_HIP(hipGetLastError());
    // every vertex pulled: merge-path tiles over the base level, then the diff level
    const Dir &R = *g->rev;
    const bool tiles = A == nullptr && g->cfg.pr_pull != 1;
    const int items = g->cfg.pr_tile == 1024 || g->cfg.pr_tile == 4096 ? g->cfg.pr_tile : MP_ITEMS;
    const bool nt = g->cfg.pr_pull != 2;
    auto tiles_kernel = items == 1024 ? (nt ? k_pr_tiles<true, 1024> : k_pr_tiles<false, 1024>)
                      : items == 4096 ? (nt ? k_pr_tiles<true, 4096> : k_pr_tiles<false, 4096>)
                                      : (nt ? k_pr_tiles<true, 2048> : k_pr_tiles<false, 2048>);
    int64_t nb = 0;
    if (tiles) {
        nb = ((int64_t)g->n + R.m + items - 1) / items;
        DG_TRY(ws.mp_row.ensure((size_t)nb + 1));
        DG_TRY(ws.mp_edge.ensure((size_t)nb + 1));
        DG_TRY(ws.mp_part.ensure(2 * (size_t)nb + 2));
        hipLaunchKernelGGL(k_mp_partition, dim3(grid_for(nb + 1)), dim3(256), 0, s, R.off.p, g->n, R.m, nb, items,
                           ws.mp_row.p, ws.mp_edge.p);
        DG_HIP(hipGetLastError());
    }
    double *pf = ws.mp_part.p, *pl = ws.mp_part.p + nb + 1;
    const double *done = prs + 3;
    // Steps are launched in groups without a host round trip; the convergence
    // test runs on the device (k_pr_reduce), and once it passes the remaining
    // launches of the group return at once.  The host reads the flag per group.
    constexpr int GROUP = 4;
    constexpr int SIDE_GROUP = 6;  // steps queued before the SSSP work starts beside them
    constexpr int AHEAD = 5;       // steps kept in flight while the host drives the SSSP rounds
    constexpr int RING = (int)(sizeof(ws.step_ev) / sizeof(ws.step_ev[0]));
    static_assert(RING > AHEAD, "the ring must hold the events of every step in flight");
    int32_t it = 0, launched = 0;
    *conv = 0;
    std::vector<std::pair<int, int>> slots;  // profiled launches of the group (pull, apply)
    // one Jacobi step (four launches: pull, rows / heavy rows, apply, reduce)
    auto launch_step = [&]() -> int {
        if (!tiles) DG_TRY(counters_clear(g));  // the heavy-row queue counters of the pull
        int ps;
        if (tiles) {
            // tiles: off 8 + xn 8 per row, col 4 + contrib 8 per base entry
            ps = prof_begin("pr_tiles", s);
            hipLaunchKernelGGL(tiles_kernel, dim3((unsigned)nb), dim3(MP_THREADS), 0, s, ws.mp_row.p, ws.mp_edge.p,
                               R.off.p, R.col.p, contrib, prs + 2, damping, xn, pf, pl, done);
            prof_end(ps, s, 16.0 * (double)g->n + 12.0 * (double)R.m);
            hipLaunchKernelGGL(k_pr_rows, dim3(grid_for(nb + R.dm)), dim3(256), 0, s, nb, items, ws.mp_row.p,
                               ws.mp_edge.p, R.off.p, pf, pl, R.dm, R.dkey.p, R.doff.p, R.dcol.p, R.keybits,
                               contrib, prs + 2, damping, xn, done);
        } else {
            int64_t blocks = std::min<int64_t>((na + 255) / 256, 65535);
            ps = prof_begin("pr_pull", s);
            hipLaunchKernelGGL(k_pr_pull, dim3((unsigned)blocks), dim3(256), 0, s, A, na, rv, contrib, prs + 2,
                               damping, xn, hq, ws.dcnt + C_HEAVY, hv, ws.dcnt + C_AUX3, heavy_deg(g),
                               heavy_deg(g), done);
            prof_end(ps, s, 28.0 * (double)na + 12.0 * (double)edges);
            hipLaunchKernelGGL(k_pr_heavy, dim3(8192), dim3(256), 0, s, rv, contrib, hq, ws.dcnt + C_HEAVY,
                               heavy_deg(g), ws.part.p);
            hipLaunchKernelGGL(k_pr_finish, dim3(64), dim3(256), 0, s, hv, ws.dcnt + C_AUX3, ws.part.p, prs + 2,
                               damping, xn);
        }
        int pa = prof_begin("pr_apply", s);
        if (tiles) {
            // the step just written becomes the current vector: no copy
            hipLaunchKernelGGL(k_pr_apply, dim3(APPLY_GROUPS), dim3(256), 0, s, A, na, xn, x, (double *)nullptr,
                               contrib, g->fwd.deg.p, partials, partials2, dprev, dprev2, prs);
            prof_end(pa, s, 28.0 * (double)na);
            std::swap(x, xn);
        } else {
            hipLaunchKernelGGL(k_pr_apply, dim3(APPLY_GROUPS), dim3(256), 0, s, A, na, xn, x, x, contrib,
                               g->fwd.deg.p, partials, partials2, dprev, dprev2, prs);
            prof_end(pa, s, 40.0 * (double)na);
        }
        hipLaunchKernelGGL(k_pr_reduce, dim3(1), dim3(256), 0, s, partials, partials2, APPLY_GROUPS, (int)global,
                           S, damping, ninv, tol, 0, extrap, prs, step_out);
        DG_HIP(hipGetLastError());
        slots.emplace_back(ps, pa);
        return DG_OK;
    };
    while (launched < max_iter && na > 0) {
        // the first group may be sized from the previous update's step count (at most
        // 64): one host round trip instead of several; launches past convergence
        // return at once.
        const bool side_waits = side && tiles && !side->done;
        int want = GROUP;
        if (launched == 0 && first_group > GROUP) want = std::min(first_group, 64);
        else if (launched > 0 && first_group > launched + GROUP) want = std::min(first_group - launched, 64);
        const int grp = std::min(want, max_iter - launched);
        slots.clear();
        int queued = 0;
        if (side_waits) {
            // Tile steps touch no state the SSSP update uses, so it runs on the second
            // stream beside them.  The host can only queue about two dozen launches
            // ahead of the device before a launch call blocks, and it drives the SSSP
            // rounds itself: so it queues SIDE_GROUP steps, starts the SSSP work, and
            // whenever it waits on the SSSP stream it queues more of the group's steps,
            // AHEAD of the last one the device has finished (events in a ring).
            for (auto &e : ws.step_ev)
                if (!e) DG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            auto queue_one = [&]() -> int {
                DG_TRY(launch_step());
                DG_HIP(hipEventRecord(ws.step_ev[queued % RING], s));
                ++queued;
                return DG_OK;
            };
            while (queued < std::min(SIDE_GROUP, grp)) DG_TRY(queue_one());
            int prc = DG_OK;
            std::function<void()> pump = [&]() {
                while (prc == DG_OK && queued < grp &&
                       (queued < AHEAD || hipEventQuery(ws.step_ev[(queued - AHEAD) % RING]) == hipSuccess))
                    prc = queue_one();
            };
            g->pump = &pump;
            side->beside = true;
            side->run();
            g->pump = nullptr;
            DG_TRY(prc);
        }
        for (; queued < grp; ++queued) DG_TRY(launch_step());
        launched += grp;
        double hp[11];
        // the host slots after the counters: a counter read of a side stream leaves them alone
        DG_HIP(hipMemcpyAsync(ws.hcnt + C_COUNT, prs, sizeof(hp), hipMemcpyDeviceToHost, s));
        DG_HIP(hipStreamSynchronize(s));
        std::memcpy(hp, ws.hcnt + C_COUNT, sizeof(hp));
        const int32_t total = (int32_t)hp[4];
        ws.pr_moves = (int32_t)hp[10];
        // launches after convergence did no work: keep them out of the timings
        for (int j = total - it; j < (int)slots.size(); ++j) {
            prof_drop(slots[j].first);
            prof_drop(slots[j].second);
        }
        it = total;
        if (hp[3] != 0.0) {
            *conv = 1;
            break;
        }
    }
    if (na == 0) *conv = 1;
    *iters = it;
    // whole-graph steps alternate the buffers: step k wrote xn if k is odd
    x = x_home;
    xn = xn_home;
    if (tiles && (it & 1)) DG_HIP(hipMemcpyAsync(x, xn, (size_t)g->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (global && na > 0) {
        hipLaunchKernelGGL(k_pr_rescale, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, x, contrib, g->fwd.deg.p,
                           prs, S, damping);
        DG_HIP(hipGetLastError());
    }
    return DG_OK;
}

// Static solve: global form from the uniform vector (S = 1).
int pr_static_solve(dg_graph *g, double damping, double tol, int32_t max_iter, double *x,
                    double *contrib, double *xn, int32_t *iters, int32_t *conv) {
    DG_TRY(ensure_pr_ws(g));
    hipLaunchKernelGGL(k_pr_init, dim3(grid_for(g->n)), dim3(256), 0, g->stream, g->n, x, contrib,
                       g->fwd.deg.p);
    DG_HIP(hipGetLastError());
    return pr_iterate(g, nullptr, g->n, g->rev->m + g->rev->dm, damping, tol, max_iter, true, 1.0, x, xn,
                      contrib, iters, conv);
}

// ---- residual push (pr_mode 3) ------------------------------------------------------
// The in-place / residual alternative to the Jacobi sweeps (the paper's
// evaluation credits in-place PageRank with faster convergence; its Dynamic PR
// listing iterates only flagged vertices).  It works on the local, dangling-dropped
// system x = (1-d)/n + d P^T x, whose residual r = (1-d)/n + d P^T x - x the query
// keeps for every vertex.  Pushing vertex v moves its residual into x[v] and hands
// d r[v] / outdeg(v) to each out-neighbour's residual, so total residual mass drops
// by at least (1 - d) r[v] per push.  After a batch, only the vertices whose
// equation changed get a new residual (heads of changed arcs and out-neighbours of
// tails whose out-degree changed); rounds push every candidate whose |r| exceeds
// theta = tol * sum(x) / (4 n) (the next candidates are the out-neighbours of the
// pushed vertices) until none does, which leaves ||r||_1 <= tol *
// sum(x) / 4 -- the Jacobi stopping rule (its L1 step is exactly ||r||_1) with
// room to spare; a final reduction confirms it.  Unlike the Jacobi sweeps, work
// stays near the batch on graphs whose residual fades before it spreads (long
// paths, no dangling mass to spread uniformly); on small-diameter graphs it
// reaches everything like the sweeps.  Sums use FP64 atomics, so the last bits
// vary from run to run (results stay within the same tolerance).

// r[v] = (1-d)/n + d * sum of contrib over live in-entries - x[v], one wave per
// vertex of L (L == nullptr: every vertex), in a fixed lane order.
__global__ __launch_bounds__(256) void k_push_resid(const int32_t *L, int64_t nl, DirView r,
                                                    const double *__restrict__ contrib, const double *x,
                                                    double damp, double base, double *res) {
    const int64_t nwaves = gstride() / WAVE;
    const int l = lane_id();
    for (int64_t i = gtid() / WAVE; i < nl; i += nwaves) {
        const int32_t v = L ? L[i] : (int32_t)i;
        double acc = 0.0;
        for (int64_t e = r.off[v] + l; e < r.off[v + 1]; e += WAVE) {
            const uint32_t c = (uint32_t)r.col[e];
            if (!(c & DEAD)) acc += contrib[c & ID_MASK];
        }
        for (int64_t e = r.doff[v] + l; e < r.doff[v + 1]; e += WAVE) {
            const uint32_t c = (uint32_t)r.dcol[e];
            if (!(c & DEAD)) acc += contrib[c & ID_MASK];
        }
        acc = wave_sum(acc);
        if (l == 0) res[v] = base + damp * acc - x[v];
    }
}

// Vertices of L (nullptr: all) with |r| > theta, appended once each (stamp st).
__global__ void k_push_select(const int32_t *L, int64_t nl, const double *res, double theta, int32_t *stamp,
                              int32_t st, int32_t *out, int64_t *count) {
    __shared__ BlockScratch sc;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nl; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        bool p = false;
        int32_t v = 0;
        if (i < nl) {
            v = L ? L[i] : (int32_t)i;
            p = fabs(res[v]) > theta && atomicExch(&stamp[v], st) != st;
        }
        const int64_t slot = block_append(count, p, sc);
        if (p) out[slot] = v;
    }
}

// Take the residual of each frontier vertex whose |r| exceeds theta into x (no
// push of this round is in flight: the expansion that adds to residuals runs
// after this launch).  The others keep their residual and push nothing (share 0).
__global__ void k_push_take(const int32_t *F, int64_t nf, double *res, double *x, double *contrib, double *share,
                            const int32_t *deg, double damp, double theta, int64_t *edges) {
    __shared__ BlockScratch sc;
    int64_t e = 0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += gstride()) {
        const int64_t i = base + threadIdx.x;
        if (i < nf) {
            const int32_t v = F[i];
            const double t = res[v];
            const int32_t dg = deg[v];
            if (fabs(t) > theta) {
                res[v] = 0.0;
                const double xv = x[v] + t;
                x[v] = xv;
                contrib[v] = dg > 0 ? xv / (double)dg : 0.0;
                share[v] = dg > 0 ? damp * t / (double)dg : 0.0;
                e += dg;
            } else {
                share[v] = 0.0;
            }
        }
    }
    block_count(edges, e, sc);
}

// Hand each pushed vertex's share to its out-neighbours (atomics whose result is
// not needed); every neighbour joins the next round's candidates (once, stamp
// st), where the take decides whether its residual is worth pushing.
struct PushOp {
    double *res;
    const double *share;
    int32_t *stamp;
    int32_t st;
    int32_t *next;
    int64_t *ncount;
    __device__ bool vtx(int32_t v, int32_t &pay) const {
        pay = 0;
        return share[v] != 0.0;
    }
    __device__ bool edge(bool valid, int32_t v, int32_t, int32_t x, int32_t) const {
        if (!valid) return false;
        unsafeAtomicAdd(&res[x], share[v]);
        // plain load first: most neighbours are already candidates
        return stamp[x] != st && atomicExch(&stamp[x], st) != st;
    }
    __device__ SinkTarget sink() const { return SinkTarget{next, ncount}; }
};

__global__ __launch_bounds__(256) void k_abs_sum(const double *x, int64_t n, double *partials) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = gtid(); i < n; i += gstride()) acc += fabs(x[i]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

static double tol_of(dg_query *q) {
    double sc = q->g->cfg.pr_tol_scale > 0 ? q->g->cfg.pr_tol_scale : 1.0;
    return q->tol * sc;
}

static int pr_mass(dg_query *q, double *S);

// sum |v| over n entries into *out (fixed block order).
static int abs_sum(dg_graph *g, const double *v, double *out) {
    hipStream_t s = g->stream;
    double *partials = g->ws.part.p;
    double *dsum = reinterpret_cast<double *>(g->ws.dcnt + C_RED0);
    hipLaunchKernelGGL(k_abs_sum, dim3(APPLY_GROUPS), dim3(256), 0, s, v, (int64_t)g->n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, APPLY_GROUPS, dsum);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    std::memcpy(out, g->ws.hcnt + C_RED0, sizeof(double));
    return DG_OK;
}

// Residual push from the residuals of L (recomputed first; L == nullptr with
// nl == n: every vertex) until no |r| exceeds theta and ||r||_1 <= tol * sum(x).
static int pr_push_run(dg_query *q, const int32_t *L, int64_t nl, dg_batch_stats *st) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    DG_TRY(ensure_pr_ws(g));
    DG_TRY(q->res.ensure((size_t)g->n + 1));
    const double d = q->damping, base = (1.0 - d) / (double)g->n;
    double S = 0.0;
    DG_TRY(pr_mass(q, &S));
    const double tol = tol_of(q) * S;
    const double theta = tol / (4.0 * (double)g->n);
    if (nl > 0)
        hipLaunchKernelGGL(k_push_resid, dim3(grid_for(nl * WAVE)), dim3(256), 0, s, L, nl, view(*g->rev),
                           q->contrib.p, q->x.p, d, base, q->res.p);
    DG_HIP(hipGetLastError());
    int32_t *F = ws.f0.p, *N = ws.f1.p;
    int32_t stamp;
    DG_TRY(next_stamp(g, &stamp));
    DG_TRY(counters_clear(g));
    if (nl > 0)
        hipLaunchKernelGGL(k_push_select, dim3(grid_for(nl)), dim3(256), 0, s, L, nl, q->res.p, theta, ws.stamp.p,
                           stamp, F, ws.dcnt + C_F0);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    int64_t nf = ws.hcnt[C_F0];
    int32_t rounds = 0, conv = 0;
    int64_t edges = 0;
    ExpandArgs a;
    a.g = view(g->fwd);
    a.hq = reinterpret_cast<int64_t *>(ws.heavy.p);
    a.hcount = ws.dcnt + C_HEAVY;
    a.heavy_deg = heavy_deg(g);
    a.chunk = heavy_deg(g);
    double *share = q->xn.p;  // scratch between calls
    for (;;) {
        while (nf > 0 && rounds < q->max_iter) {
            DG_TRY(counters_clear(g));
            const int ps = prof_begin("pr_push", s);
            hipLaunchKernelGGL(k_push_take, dim3(grid_for(nf)), dim3(256), 0, s, F, nf, q->res.p, q->x.p,
                               q->contrib.p, share, g->fwd.deg.p, d, theta, ws.dcnt + C_AUX0);
            DG_HIP(hipGetLastError());
            DG_TRY(next_stamp(g, &stamp));
            a.F = F;
            a.nf = nf;
            PushOp op{q->res.p, share, ws.stamp.p, stamp, N, ws.dcnt + C_F1};
            DG_TRY(launch_expand(s, a, op, 8192));
            DG_TRY(counters_read(g));
            // per pushed vertex: F entry 4, residual 8 read + 8 written, x 8 + 8, contrib 8, share 8,
            // degree 4 and offsets 16; per arc: col 4, residual atomic 8 + 8
            prof_end(ps, s, 0.0);
            prof_add(ps, 72.0 * (double)nf + 20.0 * (double)ws.hcnt[C_AUX0]);
            edges += ws.hcnt[C_AUX0];
            nf = ws.hcnt[C_F1];
            std::swap(F, N);
            ++rounds;
        }
        double r1 = 0.0;
        DG_TRY(abs_sum(g, q->res.p, &r1));
        DG_TRY(pr_mass(q, &S));
        if (r1 <= tol_of(q) * S) {
            conv = 1;
            break;
        }
        if (rounds >= q->max_iter) break;
        // residual left above the bound (the threshold of earlier batches differed):
        // push every vertex above theta
        DG_TRY(next_stamp(g, &stamp));
        DG_TRY(counters_clear(g));
        hipLaunchKernelGGL(k_push_select, dim3(grid_for(g->n)), dim3(256), 0, s, (const int32_t *)nullptr,
                           (int64_t)g->n, q->res.p, theta, ws.stamp.p, stamp, F, ws.dcnt + C_F0);
        DG_HIP(hipGetLastError());
        DG_TRY(counters_read(g));
        nf = ws.hcnt[C_F0];
        if (nf == 0) break;
    }
    q->last_iters = rounds;
    q->converged = conv;
    if (st) {
        st->pr_iterations += rounds;
        st->edges_traversed += edges;
    }
    return DG_OK;
}

int pr_init(dg_query *q) {
    dg_graph *g = q->g;
    DG_TRY(q->x.ensure((size_t)g->n + 1));
    DG_TRY(q->xn.ensure((size_t)g->n + 1));
    DG_TRY(q->contrib.ensure((size_t)g->n + 1));
    DG_TRY(pr_static_solve(g, q->damping, tol_of(q), q->max_iter, q->x.p, q->contrib.p, q->xn.p,
                           &q->last_iters, &q->converged));
    // residual push keeps the residual of every vertex from here on
    if (g->cfg.pr_mode == 3) {
        const int32_t it = q->last_iters;
        DG_TRY(pr_push_run(q, nullptr, g->n, nullptr));
        q->last_iters += it;
    }
    return DG_OK;
}

static int pr_update(dg_query *q, int64_t adel, int64_t ains, dg_batch_stats *st, SideWork *side);

// *S = sum(x) of the query's current values (fixed block order, so deterministic).
static int pr_mass(dg_query *q, double *S) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    const int64_t qcap = 2 * (std::max(g->fwd.m + g->fwd.dm, g->rev->m + g->rev->dm) / heavy_deg(g) + 2) +
                         g->n / 8 + 64;
    double *partials = ws.part.p + qcap;
    hipLaunchKernelGGL(k_sum_vec2, dim3(APPLY_GROUPS), dim3(256), 0, s, q->x.p, g->fwd.deg.p, (int64_t)g->n,
                       partials);
    hipLaunchKernelGGL(k_pr_reduce, dim3(1), dim3(256), 0, s, partials, partials, APPLY_GROUPS, 0, 0.0, q->damping,
                       1.0, 0.0, 1, 0, ws.prs.p, ws.prs.p + 5);
    DG_HIP(hipGetLastError());
    // prs[0] here holds the plain sum (first partial of each pair)
    DG_HIP(hipMemcpyAsync(ws.hcnt + C_COUNT, ws.prs.p, sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    std::memcpy(S, ws.hcnt + C_COUNT, sizeof(double));
    return DG_OK;
}

int pr_post_update(dg_query *q, int64_t adel, int64_t ains, dg_batch_stats *st, SideWork *side) {
    const int rc = pr_update(q, adel, ains, st, side);
    if (side) {
        side->run();  // not yet run if the steps could not overlap it
        if (rc == DG_OK) return side->rc;
    }
    return rc;
}

static int pr_update(dg_query *q, int64_t adel, int64_t ains, dg_batch_stats *st, SideWork *side) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    Work &ws = g->ws;
    if (adel + ains == 0) {
        q->last_iters = 0;
        return DG_OK;
    }
    DG_TRY(ensure_pr_ws(g));
    const int64_t qcap = 2 * (std::max(g->fwd.m + g->fwd.dm, g->rev->m + g->rev->dm) / heavy_deg(g) + 2) +
                         g->n / 8 + 64;
    int64_t *hq = reinterpret_cast<int64_t *>(ws.heavy.p);
    int32_t *Alist = ws.f0.p;
    int32_t *S = ws.f1.p;
    // tails of changed arcs (distinct)
    int32_t st_s, st_a;
    DG_TRY(next_stamp(g, &st_s));
    DG_TRY(counters_clear(g));
    if (adel > 0)
        hipLaunchKernelGGL(k_mark_list, dim3(grid_for(adel)), dim3(256), 0, s, adel, ws.adu.p,
                           ws.stamp.p, st_s, S, ws.dcnt + C_AUX0);
    if (ains > 0)
        hipLaunchKernelGGL(k_mark_list, dim3(grid_for(ains)), dim3(256), 0, s, ains, ws.aiu.p,
                           ws.stamp.p, st_s, S, ws.dcnt + C_AUX0);
    // the tails' share x / outdeg changed: refresh it before any Jacobi step (the
    // count of distinct tails stays on the device; grids sized for every changed arc)
    hipLaunchKernelGGL(k_refresh_contrib, dim3(grid_for(adel + ains)), dim3(256), 0, s, ws.dcnt + C_AUX0, S,
                       q->x.p, g->fwd.deg.p, q->contrib.p);
    const int mode = g->cfg.pr_mode;  // 0 auto, 1 local, 2 global, 3 residual push
    const int64_t vlimit = (int64_t)(0.2 * (double)g->n);
    bool global = mode == 2;
    // the seeds are the heads plus the tails' out-neighbours; when their count with
    // repeats already passes 20% of the vertices, the automatic mode takes the global
    // form without expanding (both forms reach the same ranks; this only picks the
    // cheaper one).  One read brings the tail count and that sum.
    if (mode == 0)
        hipLaunchKernelGGL(k_sum_degrees, dim3(grid_for(adel + ains)), dim3(256), 0, s, S, (int64_t)0,
                           ws.dcnt + C_AUX0, g->fwd.off.p, g->fwd.doff.p, ws.dcnt + C_AUX1);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    const int64_t ns = ws.hcnt[C_AUX0];
    if (mode == 0 && adel + ains + ws.hcnt[C_AUX1] >= vlimit) global = true;
    int64_t na = 0;
    ExpandArgs a;
    a.g = view(g->fwd);
    a.hq = hq;
    a.hcount = ws.dcnt + C_HEAVY;
    a.heavy_deg = heavy_deg(g);
    a.chunk = heavy_deg(g);
    (void)qcap;
    if (!global) {
        // seeds: heads of changed arcs, then all out-neighbours of the tails
        DG_TRY(next_stamp(g, &st_a));
        DG_TRY(counters_clear(g));
        if (adel > 0)
            hipLaunchKernelGGL(k_mark_list, dim3(grid_for(adel)), dim3(256), 0, s, adel, ws.adv.p,
                               ws.stamp.p, st_a, Alist, ws.dcnt + C_F0);
        if (ains > 0)
            hipLaunchKernelGGL(k_mark_list, dim3(grid_for(ains)), dim3(256), 0, s, ains, ws.aiv.p,
                               ws.stamp.p, st_a, Alist, ws.dcnt + C_F0);
        DG_HIP(hipGetLastError());
        DG_TRY(counters_read(g));
        na = ws.hcnt[C_F0];
        DG_TRY(counters_clear(g));
        a.F = S;
        a.nf = ns;
        ReachOp op{ws.stamp.p, st_a, Alist + na, ws.dcnt + C_F1};
        DG_TRY(launch_expand(s, a, op, 8192));
        DG_TRY(counters_read(g));
        na += ws.hcnt[C_F1];
        if (mode == 3) {
            // residual push from the seeds instead of the reach closure and sweeps
            DG_TRY(pr_push_run(q, Alist, na, st));
            if (st) st->pr_affected += na;
            return DG_OK;
        }
        if (mode == 0 && na >= vlimit) global = true;
    }
    // forward closure (propagateNodeFlags): levels appended to Alist.  In the
    // automatic mode it stops once the set passes 20% of the vertices, since the
    // global form then runs over every vertex anyway.
    int64_t lo = 0, hi = na;
    while (!global && hi > lo) {
        DG_TRY(counters_clear(g));
        a.F = Alist + lo;
        a.nf = hi - lo;
        ReachOp op{ws.stamp.p, st_a, Alist + hi, ws.dcnt + C_F1};
        DG_TRY(launch_expand(s, a, op, 8192));
        DG_TRY(counters_read(g));
        lo = hi;
        hi += ws.hcnt[C_F1];
        if (mode == 0 && hi >= vlimit) global = true;
    }
    na = hi;
    int64_t edges = 0;
    const int64_t all_edges = g->rev->m + g->rev->dm;
    if (!global && na > 0) {
        DG_TRY(ws.scan64.ensure(2 * ((size_t)g->n + 1)));
        int64_t *flags = ws.scan64.p, *pos = ws.scan64.p + (g->n + 1);
        hipLaunchKernelGGL(k_stamp_flags, dim3(grid_for(g->n + 1)), dim3(256), 0, s, g->n, ws.stamp.p, st_a,
                           flags);
        DG_TRY(scan_excl(g, flags, pos, g->n + 1));
        hipLaunchKernelGGL(k_compact_flags, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, flags, pos, Alist);
        DG_TRY(counters_clear(g));
        hipLaunchKernelGGL(k_sum_degrees, dim3(grid_for(na)), dim3(256), 0, s, Alist, na, (const int64_t *)nullptr,
                           g->rev->off.p, g->rev->doff.p, ws.dcnt + C_AUX0);
        DG_HIP(hipGetLastError());
        DG_TRY(counters_read(g));
        edges = ws.hcnt[C_AUX0];
        if (mode == 0 && (double)edges >= 0.2 * (double)all_edges) global = true;
    }
    int32_t iters = 0, conv = 0;
    // S = sum(x) of the warm start.  Both forms stop on the L1 step of the
    // normalised ranks x / S, so the tolerance on x is tol * S (the global form
    // also conserves S).
    // (S = -1: the mass stays on the device, summed by the iteration's set-up)
    if (global) {
        na = g->n;
        edges = all_edges;
        DG_TRY(pr_iterate(g, nullptr, na, edges, q->damping, tol_of(q), q->max_iter, true, -1.0, q->x.p, q->xn.p,
                          q->contrib.p, &iters, &conv, side, q->last_iters));
    } else {
        DG_TRY(pr_iterate(g, Alist, na, edges, q->damping, tol_of(q), q->max_iter, false, -1.0, q->x.p, q->xn.p,
                          q->contrib.p, &iters, &conv));
    }
    q->last_iters = iters;
    q->converged = conv;
    if (st) {
        st->pr_iterations += iters;
        st->pr_moves += g->ws.pr_moves;
        st->pr_affected += na;
        st->edges_traversed += edges * iters;
    }
    return DG_OK;
}

// rank = x / sum(x), written to device memory (dev) or copied to the host.
int pr_normalize(dg_graph *g, const double *x, double *rank, bool dev) {
    hipStream_t s = g->stream;
    DG_TRY(ensure_pr_ws(g));
    double *partials = g->ws.part.p;
    double *dsum = reinterpret_cast<double *>(g->ws.dcnt + C_RED0);
    const int32_t *perm = g->relabeled ? g->perm.p : nullptr;
    hipLaunchKernelGGL(k_sum_vec, dim3(APPLY_GROUPS), dim3(256), 0, s, x, (int64_t)g->n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, APPLY_GROUPS, dsum);
    DG_HIP(hipGetLastError());
    if (dev) {
        hipLaunchKernelGGL(k_scale, dim3(grid_for(g->n)), dim3(256), 0, s, x, perm, (int64_t)g->n, dsum, rank);
        DG_HIP(hipGetLastError());
        DG_HIP(hipStreamSynchronize(s));
        return DG_OK;
    }
    DBuf<double> &tmp = g->ws.rbuf;
    DG_TRY(tmp.ensure((size_t)g->n + 1));
    hipLaunchKernelGGL(k_scale, dim3(grid_for(g->n)), dim3(256), 0, s, x, perm, (int64_t)g->n, dsum, tmp.p);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(rank, tmp.p, (size_t)g->n * sizeof(double), hipMemcpyDeviceToHost, s);
    hipError_t e3 = hipStreamSynchronize(s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return set_error(DG_EDEVICE, "pagerank read failed");
    return DG_OK;
}

int pr_read(dg_query *q, double *rank, bool dev) { return pr_normalize(q->g, q->x.p, rank, dev); }

// ---- reading ranks without allocating -------------------------------------------------
// The same normalisation as pr_normalize, for callers that cannot allocate device
// memory: the partial sums, their total and the staging of a host copy live in a
// fixed array in device memory, one copy per GPU, held until the process ends.
// Layout (doubles): [0, APPLY_GROUPS) partial sums, [APPLY_GROUPS] the total,
// [NOALLOC_STAGE, NOALLOC_DOUBLES) staging of a host copy.
constexpr int64_t NOALLOC_DOUBLES = 1 << 19;  // 4 MiB
constexpr int64_t NOALLOC_STAGE = 2048;
static_assert(NOALLOC_DOUBLES - NOALLOC_STAGE == DG_NOALLOC_MAX_HOST_N, "header limit matches the scratch");
static_assert(APPLY_GROUPS + 1 <= NOALLOC_STAGE, "partials fit below the staging area");
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;       // one call at a time per process: calls share the array
static double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device, with
// that device current; the array's host-side name is not a device address).
static int scratch_of_current_device(double **out) {
    int dev = 0;
    DG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(DG_EDEVICE, "device %d beyond the scratch table", dev);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(DG_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return DG_OK;
}

int pr_read_noalloc(dg_query *q, double *rank, bool dev) {
    dg_graph *g = q->g;
    if (!dev && (int64_t)g->n > DG_NOALLOC_MAX_HOST_N)
        return set_error(DG_EINVAL, "no-allocation read into host memory holds at most %lld ranks (n = %d); pass "
                                    "a device buffer with DG_DEVICE_PTRS",
                         (long long)DG_NOALLOC_MAX_HOST_N, g->n);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    double *sp = nullptr;
    DG_TRY(scratch_of_current_device(&sp));
    hipStream_t s = g->stream;
    const int32_t *perm = g->relabeled ? g->perm.p : nullptr;
    // every slot the kernels read is written first in this call (partials by
    // k_sum_vec, the total by k_sum_partials), so nothing needs clearing
    hipLaunchKernelGGL(k_sum_vec, dim3(APPLY_GROUPS), dim3(256), 0, s, q->x.p, (int64_t)g->n, sp);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, sp, APPLY_GROUPS, sp + APPLY_GROUPS);
    double *out = dev ? rank : sp + NOALLOC_STAGE;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(g->n)), dim3(256), 0, s, q->x.p, perm, (int64_t)g->n,
                       sp + APPLY_GROUPS, out);
    DG_HIP(hipGetLastError());
    if (!dev) DG_HIP(hipMemcpyAsync(rank, out, (size_t)g->n * sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    return DG_OK;
}

// ---- checkpoint / resume -----------------------------------------------------------------
// The exported state is x itself (the dangling-dropped system's unnormalised
// values) in the caller's vertex order.  An import takes any non-negative finite x
// as a warm start and runs the global form until the L1 step meets the tolerance,
// so a state exported from this graph resumes after one confirming step, and any
// other start still converges to the same ranks.

// x[perm[c]] = X[c], contrib = x / outdeg; *bad counts negative or non-finite values.
__global__ void k_pr_import(int32_t n, const double *X, const int32_t *perm, const int32_t *deg, double *x,
                            double *contrib, int64_t *bad) {
    int64_t nbad = 0;
    for (int64_t c = gtid(); c < n; c += gstride()) {
        double v = X[c];
        if (!(v >= 0.0 && v <= 1.0e300)) {
            ++nbad;
            v = 0.0;
        }
        const int64_t i = perm ? perm[c] : c;
        x[i] = v;
        contrib[i] = deg[i] > 0 ? v / (double)deg[i] : 0.0;
    }
    nbad = wave_sum(nbad);
    if (lane_id() == 0 && nbad) atomicAdd((unsigned long long *)bad, (unsigned long long)nbad);
}

__global__ void k_pr_export(int32_t n, const double *x, const int32_t *perm, double *X) {
    for (int64_t c = gtid(); c < n; c += gstride()) X[c] = x[perm ? perm[c] : c];
}

int pr_export(dg_query *q, double *xh) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    DG_TRY(g->ws.rbuf.ensure((size_t)g->n + 1));
    hipLaunchKernelGGL(k_pr_export, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, q->x.p,
                       g->relabeled ? (const int32_t *)g->perm.p : nullptr, g->ws.rbuf.p);
    DG_HIP(hipGetLastError());
    DG_HIP(hipMemcpyAsync(xh, g->ws.rbuf.p, (size_t)g->n * sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    return DG_OK;
}

int pr_import(dg_query *q, const double *xh) {
    dg_graph *g = q->g;
    hipStream_t s = g->stream;
    DG_TRY(q->x.ensure((size_t)g->n + 1));
    DG_TRY(q->xn.ensure((size_t)g->n + 1));
    DG_TRY(q->contrib.ensure((size_t)g->n + 1));
    DG_TRY(ensure_pr_ws(g));
    DG_TRY(g->ws.rbuf.ensure((size_t)g->n + 1));
    DG_HIP(hipMemcpyAsync(g->ws.rbuf.p, xh, (size_t)g->n * sizeof(double), hipMemcpyHostToDevice, s));
    DG_TRY(counters_clear(g));
    hipLaunchKernelGGL(k_pr_import, dim3(grid_for(g->n)), dim3(256), 0, s, g->n, g->ws.rbuf.p,
                       g->relabeled ? (const int32_t *)g->perm.p : nullptr, g->fwd.deg.p, q->x.p, q->contrib.p,
                       g->ws.dcnt + C_AUX0);
    DG_HIP(hipGetLastError());
    DG_TRY(counters_read(g));
    if (g->ws.hcnt[C_AUX0] != 0)
        return set_error(DG_EINVAL, "imported PageRank state: %lld negative or non-finite values",
                         (long long)g->ws.hcnt[C_AUX0]);
    double Ssum = 0.0;
    DG_TRY(pr_mass(q, &Ssum));
    if (!(Ssum > 0.0)) return set_error(DG_EINVAL, "imported PageRank state sums to zero");
    int32_t iters = 0, conv = 0;
    DG_TRY(pr_iterate(g, nullptr, g->n, g->rev->m + g->rev->dm, q->damping, tol_of(q) * Ssum, q->max_iter, true,
                      Ssum, q->x.p, q->xn.p, q->contrib.p, &iters, &conv));
    q->last_iters = iters;
    q->converged = conv;
    if (g->cfg.pr_mode == 3) {
        DG_TRY(pr_push_run(q, nullptr, g->n, nullptr));
        q->last_iters += iters;
    }
    return DG_OK;
}



}  // namespace dg
