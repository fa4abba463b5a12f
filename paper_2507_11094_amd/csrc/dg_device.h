// Device-side helpers shared by the kernels (64-wide CDNA wavefronts).
#pragma once

#include <type_traits>

#include "dg_internal.h"

namespace dg {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// Position of neighbour v in the sorted base row, or -1.  Tombstoned entries
// keep their place in the order, so they are found too (caller checks flags).
__device__ __forceinline__ int64_t find_sorted(const int32_t *__restrict__ col, int64_t lo,
                                               int64_t hi, uint32_t v) {
    int64_t end = hi;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        uint32_t c = (uint32_t)col[mid] & ID_MASK;
        if (c < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo < end && ((uint32_t)col[lo] & ID_MASK) == v) return lo;
    return -1;
}

// First position in [lo, hi) whose neighbour id is >= v.
__device__ __forceinline__ int64_t lower_sorted(const int32_t *__restrict__ col, int64_t lo,
                                                int64_t hi, uint32_t v) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (((uint32_t)col[mid] & ID_MASK) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t lower_key(const uint64_t *__restrict__ k, int64_t lo, int64_t hi,
                                             uint64_t v) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (k[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Searches for items q0 .. q0+K-1 of an N-item chunk, run in lockstep so that a
// lane keeps K loads in flight instead of one: for each item with act[q], v[q] is
// looked up in the sorted range [off[row[q]], off[row[q] + 1]) of col, and out[q]
// is its position (flags ignored, so tombstones are found too) or -1.
template <int K, int N>
__device__ __forceinline__ void find_rows_k(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                            const int32_t (&row)[N], const uint32_t (&v)[N],
                                            const bool (&act)[N], int64_t (&out)[N], int q0) {
    int64_t lo[K], hi[K], end[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        lo[j] = act[q0 + j] ? off[row[q0 + j]] : 0;
        end[j] = act[q0 + j] ? off[row[q0 + j] + 1] : 0;
        hi[j] = end[j];
    }
    for (;;) {
        uint32_t c[K];
#pragma unroll
        for (int j = 0; j < K; ++j) c[j] = lo[j] < hi[j] ? ((uint32_t)col[(lo[j] + hi[j]) >> 1] & ID_MASK) : 0u;
        bool more = false;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (lo[j] < hi[j]) {
                const int64_t mid = (lo[j] + hi[j]) >> 1;
                if (c[j] < v[q0 + j]) lo[j] = mid + 1;
                else hi[j] = mid;
            }
            more |= lo[j] < hi[j];
        }
        if (!more) break;
    }
    uint32_t c[K];
#pragma unroll
    for (int j = 0; j < K; ++j) c[j] = lo[j] < end[j] ? ((uint32_t)col[lo[j]] & ID_MASK) : ~0u;
#pragma unroll
    for (int j = 0; j < K; ++j) out[q0 + j] = lo[j] < end[j] && c[j] == v[q0 + j] ? lo[j] : -1;
}

// Base level, then the diff level for the items the base level lacks, K at a time.
constexpr int FIND_K = 4;
template <int N>
__device__ __forceinline__ void find_arcs(const int64_t *off, const int32_t *col, const int64_t *doff,
                                          const int32_t *dcol, const int32_t (&row)[N], const uint32_t (&v)[N],
                                          const bool (&act)[N], int64_t (&pb)[N], int64_t (&pd)[N]) {
#pragma unroll
    for (int h = 0; h < N; h += FIND_K) find_rows_k<FIND_K>(off, col, row, v, act, pb, h);
    bool miss[N];
#pragma unroll
    for (int q = 0; q < N; ++q) miss[q] = act[q] && pb[q] < 0;
#pragma unroll
    for (int h = 0; h < N; h += FIND_K) find_rows_k<FIND_K>(doff, dcol, row, v, miss, pd, h);
}

// Largest r in [lo, hi] with off[r] <= i: the row holding entry i.
__device__ __forceinline__ int32_t row_of(const int64_t *__restrict__ off, int32_t lo, int32_t hi,
                                          int64_t i) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Orders the LDS writes of a wave's lanes before the reads that follow (all lanes
// of the wave must reach it).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP lane moves (the data-parallel-primitive operand modifier of gfx9 VALU
// instructions): lane i receives the value of another lane without going through
// LDS.  Controls used here: row_shr:k (0x110 + k; from lane i - k of the same
// 16-lane row), row_bcast:15 (0x142; lane 15 of a row into every lane of the next
// row) and row_bcast:31 (0x143; lane 31 into rows 2 and 3).  Lanes of rows
// outside ROW_MASK, and lanes whose source is outside the row when BOUND_ZERO is
// set, receive 0.  Every lane of the wave must be active.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, BOUND_ZERO);
}
template <int CTRL, int ROW_MASK, bool BOUND_ZERO, class T>
__device__ __forceinline__ T dpp_move(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit integers");
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = (uint64_t)x;
        const uint64_t lo = dpp_u32<CTRL, ROW_MASK, BOUND_ZERO>((uint32_t)u);
        const uint64_t hi = dpp_u32<CTRL, ROW_MASK, BOUND_ZERO>((uint32_t)(u >> 32));
        return (T)((hi << 32) | lo);
    } else {
        return (T)dpp_u32<CTRL, ROW_MASK, BOUND_ZERO>((uint32_t)x);
    }
}

// Wave-wide inclusive scan of integers: Hillis-Steele inside each 16-lane row by
// DPP row shifts, then the row totals carried across rows by the two DPP row
// broadcasts.  Six DPP moves per 32 bits, no LDS traffic.  All lanes must be active.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    static_assert(std::is_integral<T>::value, "integer scan");
    x += dpp_move<0x111, 0xf, true>(x);   // row_shr:1
    x += dpp_move<0x112, 0xf, true>(x);   // row_shr:2
    x += dpp_move<0x114, 0xf, true>(x);   // row_shr:4
    x += dpp_move<0x118, 0xf, true>(x);   // row_shr:8
    x += dpp_move<0x142, 0xa, false>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xc, false>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

template <class T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        T y = __shfl_xor(x, d, WAVE);
        x = y < x ? y : x;
    }
    return x;
}

template <class T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        T y = __shfl_xor(x, d, WAVE);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        int32_t y = __shfl_xor(x, d, WAVE);
        x = y > x ? y : x;
    }
    return x;
}

// One atomic per wave for a counter bump of `pred` lanes; returns the slot of
// this lane (valid where pred is true).
__device__ __forceinline__ int64_t wave_append(int64_t *counter, bool pred) {
    uint64_t b = ballot(pred);
    if (b == 0) return -1;
    int leader = __ffsll((long long)b) - 1;
    int64_t base = 0;
    if (lane_id() == leader) base = atomicAdd((unsigned long long *)counter, (unsigned long long)__popcll(b));
    base = __shfl(base, leader, WAVE);
    return base + __popcll(b & lanemask_lt());
}


// ---- block-aggregated counters ------------------------------------------------------
// Atomics on one address serialise (tens of ns each), so kernels over millions of
// elements take their output slots once per block and chunk instead of once per
// wave: every thread handles CH_IPT consecutive elements, the block scans the
// per-thread counts in LDS and one thread reserves the block's total.  All
// threads of the block (blockDim == CH_T) must make the same calls.
constexpr int CH_T = 256;
constexpr int CH_IPT = 8;
constexpr int CH = CH_T * CH_IPT;

struct BlockScratch {
    int64_t w[CH_T / WAVE];
    int64_t base;
};

// Exclusive prefix of v over the block (thread order); *total = block sum.
__device__ __forceinline__ int64_t block_scan_excl(int64_t v, int64_t *total, BlockScratch &s) {
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    const int64_t incl = wave_incl_scan(v);
    if (l == WAVE - 1) s.w[wv] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < CH_T / WAVE; ++q) {
        const int64_t x = s.w[q];
        if (q < wv) before += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// First of v consecutive slots of `counter` for this thread (one atomic per block).
__device__ __forceinline__ int64_t block_reserve(int64_t *counter, int64_t v, BlockScratch &s) {
    int64_t tot;
    const int64_t ex = block_scan_excl(v, &tot, s);
    if (threadIdx.x == 0)
        s.base = tot > 0 ? (int64_t)atomicAdd((unsigned long long *)counter, (unsigned long long)tot) : 0;
    __syncthreads();
    const int64_t r = s.base + ex;
    __syncthreads();
    return r;
}

// Slot of a true predicate (one atomic per block and call; all threads call).
__device__ __forceinline__ int64_t block_append(int64_t *counter, bool pred, BlockScratch &s) {
    return block_reserve(counter, pred ? 1 : 0, s);
}

// counter += sum of v over the block (one atomic per block).
__device__ __forceinline__ void block_count(int64_t *counter, int64_t v, BlockScratch &s) {
    int64_t tot;
    (void)block_scan_excl(v, &tot, s);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)counter, (unsigned long long)tot);
}

__device__ __forceinline__ uint64_t sssp_pack(int32_t dist, int32_t parent) {
    return ((uint64_t)(uint32_t)dist << 32) | (uint64_t)(uint32_t)parent;
}
__device__ __forceinline__ int32_t sssp_dist(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ int32_t sssp_parent(uint64_t k) { return (int32_t)(uint32_t)(k & 0xffffffffu); }

// Grid-stride helpers
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

}  // namespace dg
