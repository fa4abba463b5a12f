// Frontier expansion shared by the traversals (SSSP push, subtree invalidation,
// decremental pull, PageRank reach closure).
//
// A wave takes 64 frontier vertices, scans their degrees (base row + diff row)
// with a 64-lane prefix sum and then walks the concatenated edge slots 64 at a
// time, so every lane always has an edge regardless of the degree mix (a
// load-balanced search inside the wave).  Vertices with more than `heavy_deg`
// edges are not expanded in place: they are cut into chunks of `chunk` edges that
// a second kernel spreads over the whole grid, one wave per chunk.
#pragma once

#include "dg_device.h"

namespace dg {

struct DirView {
    const int64_t *off;
    const int32_t *col;
    const int32_t *w;
    const int64_t *doff;
    const int32_t *dcol;
    const int32_t *dw;
};

inline DirView view(const Dir &d) { return DirView{d.off.p, d.col.p, d.w.p, d.doff.p, d.dcol.p, d.dw.p}; }

struct ExpandArgs {
    const int32_t *F;   // frontier
    int64_t nf;
    const int64_t *nfp = nullptr;  // when set, the frontier length is read from device memory
    DirView g;
    int64_t *hq;        // heavy chunk queue: (v << 32) | chunk
    int64_t *hcount;    // its length
    int heavy_deg;
    int chunk;
    int64_t *tally = nullptr;  // when set: += entries of the rows this step walks (traversal tally)
};

// Output of an expansion: vertices the op selects go to `out` (and `out2`, when
// set) with their lengths in `count` / `count2`.
struct SinkTarget {
    int32_t *out = nullptr;
    int64_t *count = nullptr;
    int32_t *out2 = nullptr;
    int64_t *count2 = nullptr;
};

// Per-wave staging of selected vertices in LDS: one atomic per WB_CAP entries
// instead of one per 64-edge step (same-address atomics serialise).
constexpr int WB_CAP = 256;
struct WaveSink {
    int32_t *buf;
    int n;
    SinkTarget t;
    __device__ __forceinline__ void flush() {
        if (n == 0) return;
        __builtin_amdgcn_wave_barrier();
        int64_t b1 = 0, b2 = 0;
        if (lane_id() == 0) {
            b1 = (int64_t)atomicAdd((unsigned long long *)t.count, (unsigned long long)n);
            if (t.out2) b2 = (int64_t)atomicAdd((unsigned long long *)t.count2, (unsigned long long)n);
        }
        b1 = __shfl(b1, 0, WAVE);
        b2 = __shfl(b2, 0, WAVE);
        for (int j = lane_id(); j < n; j += WAVE) {
            const int32_t x = buf[j];
            t.out[b1 + j] = x;
            if (t.out2) t.out2[b2 + j] = x;
        }
        __builtin_amdgcn_wave_barrier();
        n = 0;
    }
    __device__ __forceinline__ void push(bool p, int32_t x) {
        const uint64_t m = ballot(p);
        const int c = __popcll(m);
        if (c == 0) return;
        if (n + c > WB_CAP) flush();
        if (p) buf[n + __popcll(m & lanemask_lt())] = x;
        n += c;
    }
};

// Op interface:
//   __device__ bool vtx(int32_t v, int32_t &payload)  -- false: skip v
//   __device__ bool edge(bool valid, int32_t v, int32_t payload, int32_t x, int32_t w)
//        -- true: x goes to the op's sink
//   __device__ SinkTarget sink() const                 -- out == nullptr: no output
// edge() is called by every lane of the wave in lock-step (valid marks real edges).
template <class Op>
__global__ __launch_bounds__(256) void k_expand(ExpandArgs a, Op op) {
    __shared__ int32_t s_sink[256 / WAVE][WB_CAP];
    WaveSink sk{s_sink[threadIdx.x / WAVE], 0, op.sink()};
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    const int64_t nf = a.nfp ? *a.nfp : a.nf;
    int64_t walked = 0;  // entries of this lane's rows (heavy rows too, walked by k_expand_heavy)
    for (int64_t wb = wave_global * WAVE; wb < nf; wb += nwaves * WAVE) {
        const int64_t fi = wb + l;
        int32_t v = -1, pay = 0;
        int64_t ob = 0, od = 0;
        int32_t db = 0, tot = 0;
        if (fi < nf) {
            v = a.F[fi];
            if (op.vtx(v, pay)) {
                ob = a.g.off[v];
                db = (int32_t)(a.g.off[v + 1] - ob);
                od = a.g.doff[v];
                tot = db + (int32_t)(a.g.doff[v + 1] - od);
            }
        }
        walked += tot;
        // split heavy vertices into grid-wide chunks
        const bool heavy = tot > a.heavy_deg;
        int32_t nch = heavy ? (tot + a.chunk - 1) / a.chunk : 0;
        int64_t incl_ch = wave_incl_scan((int64_t)nch);
        int64_t tot_ch = __shfl(incl_ch, WAVE - 1, WAVE);
        int64_t base_ch = 0;
        if (l == 0 && tot_ch > 0) base_ch = atomicAdd((unsigned long long *)a.hcount, (unsigned long long)tot_ch);
        base_ch = __shfl(base_ch, 0, WAVE);
        for (int32_t c = 0; c < nch; ++c)
            a.hq[base_ch + incl_ch - nch + c] = ((int64_t)v << 32) | (uint32_t)c;
        if (heavy) tot = 0;
        // load-balanced walk over the light vertices' edges
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
            const int32_t vo = __shfl(v, o, WAVE);
            const int32_t po = __shfl(pay, o, WAVE);
            const int64_t obo = __shfl(ob, o, WAVE);
            const int64_t odo = __shfl(od, o, WAVE);
            const int32_t dbo = __shfl(db, o, WAVE);
            const int64_t exo = __shfl(excl, o, WAVE);
            bool valid = e < T;
            int32_t x = 0, wt = 0;
            if (valid) {
                int64_t j = e - exo;
                uint32_t c;
                if (j < dbo) { c = (uint32_t)a.g.col[obo + j]; wt = a.g.w ? a.g.w[obo + j] : 0; }
                else { c = (uint32_t)a.g.dcol[odo + (j - dbo)]; wt = a.g.dw ? a.g.dw[odo + (j - dbo)] : 0; }
                valid = !(c & DEAD);
                x = (int32_t)(c & ID_MASK);
            }
            const bool p = op.edge(valid, vo, po, x, wt);
            if (sk.t.out) sk.push(p, x);
        }
    }
    if (sk.t.out) sk.flush();
    if (a.tally) {  // uniform: one add per block
        __shared__ int64_t s_walked[256 / WAVE];
        walked = wave_sum(walked);
        if (l == 0) s_walked[threadIdx.x / WAVE] = walked;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < 256 / WAVE; ++w) t += s_walked[w];
            if (t) atomicAdd((unsigned long long *)a.tally, (unsigned long long)t);
        }
    }
}

// One wave per heavy chunk (grid-stride over the queue).
template <class Op>
__global__ __launch_bounds__(256) void k_expand_heavy(ExpandArgs a, Op op) {
    __shared__ int32_t s_sink[256 / WAVE][WB_CAP];
    WaveSink sk{s_sink[threadIdx.x / WAVE], 0, op.sink()};
    const int64_t wave_global = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    const int64_t nq = *a.hcount;
    for (int64_t qi = wave_global; qi < nq; qi += nwaves) {
        const int64_t ent = a.hq[qi];
        const int32_t v = (int32_t)(ent >> 32);
        const int32_t c = (int32_t)(ent & 0xffffffff);
        int32_t pay = 0;
        if (!op.vtx(v, pay)) continue;  // uniform across the wave
        const int64_t ob = a.g.off[v];
        const int32_t db = (int32_t)(a.g.off[v + 1] - ob);
        const int64_t od = a.g.doff[v];
        const int32_t tot = db + (int32_t)(a.g.doff[v + 1] - od);
        const int64_t s = (int64_t)c * a.chunk;
        const int64_t e = min((int64_t)tot, s + a.chunk);
        for (int64_t jb = s; jb < e; jb += WAVE) {
            const int64_t j = jb + l;
            bool valid = j < e;
            int32_t x = 0, wt = 0;
            if (valid) {
                uint32_t cc;
                if (j < db) { cc = (uint32_t)a.g.col[ob + j]; wt = a.g.w ? a.g.w[ob + j] : 0; }
                else { cc = (uint32_t)a.g.dcol[od + (j - db)]; wt = a.g.dw ? a.g.dw[od + (j - db)] : 0; }
                valid = !(cc & DEAD);
                x = (int32_t)(cc & ID_MASK);
            }
            const bool p = op.edge(valid, v, pay, x, wt);
            if (sk.t.out) sk.push(p, x);
        }
    }
    if (sk.t.out) sk.flush();
}

// Host side: run one expansion step of `op` over frontier F (nf entries).
// hcount must point at a zeroed device counter.  heavy_deg = NO_HEAVY: no row is
// cut into chunks (every row is walked by k_expand) and the chunk kernel is not
// launched.
constexpr int NO_HEAVY = 0x7fffffff;
template <class Op>
inline int launch_expand(hipStream_t s, const ExpandArgs &a, const Op &op, int heavy_groups) {
    if (!a.nfp && a.nf <= 0) return DG_OK;
    int64_t blocks = a.nfp ? 4096 : (a.nf + 255) / 256;  // device-side count: fixed grid-stride grid
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_expand<Op>, dim3((unsigned)blocks), dim3(256), 0, s, a, op);
    if (a.heavy_deg != NO_HEAVY)
        hipLaunchKernelGGL(k_expand_heavy<Op>, dim3(heavy_groups), dim3(256), 0, s, a, op);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(DG_EDEVICE, "expand launch failed: %s", hipGetErrorString(e));
    return DG_OK;
}

}  // namespace dg
