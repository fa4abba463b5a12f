// Sorting and prefix sums for the batch canonicalisation, the diff-level rebuild,
// the CSR merge and the compactions: an LSD radix sort of (uint64 key, int32
// value) pairs and an exclusive scan of int64, both single-pass per digit /
// call with decoupled look-back between tiles.
//
// Radix sort (8-bit digits, least significant first, stable):
//   1. one launch reads the keys once and builds the digit histogram of every
//      pass (per-wave LDS histograms), then adds them to global counts;
//   2. one launch per pass: a workgroup takes the next tile of 2,048 keys (tile
//      ids from an atomic counter, so every earlier tile is already running),
//      ranks its keys stably inside the tile (ballot match per wave, per-wave
//      digit counters in LDS), publishes its per-digit counts, looks back over
//      earlier tiles' published counts (per digit, 16 predecessors per read) to
//      find where its keys go, and scatters them through an LDS staging copy so
//      that runs of one digit are written contiguously.  Each workgroup turns
//      the pass's global counts into digit starts itself (a 256-entry scan).
// Look-back words hold a 2-bit flag (count of this tile only / inclusive prefix),
// a 14-bit epoch and a 48-bit value.  Each pass or scan takes a new epoch, so
// words left by earlier passes read as "not ready" without clearing; the array is
// cleared when the epoch wraps or the workspace is reallocated.  Every wait is
// bounded (a spin limit sets an error bit and lets the tile finish), so every
// workgroup exits.
#include <algorithm>

#include "dg_device.h"

namespace dg {

constexpr int RS_BITS = 8;
constexpr int RS_RADIX = 1 << RS_BITS;
constexpr int RS_THREADS = 256;  // four waves; thread d also owns digit d
constexpr int RS_WAVES = RS_THREADS / WAVE;
constexpr int RS_ITEMS = 8;      // keys per lane per tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_MAX_PASSES = 8;
static_assert(RS_RADIX == RS_THREADS, "one thread per digit");

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;     // int64 per lane per tile
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

constexpr uint64_t LB_AGG = 1ull << 62;   // the tile's own count
constexpr uint64_t LB_PRE = 2ull << 62;   // inclusive prefix through the tile
constexpr uint64_t LB_FLAGS = 3ull << 62;
constexpr int LB_EPOCH_SHIFT = 48;
constexpr uint64_t LB_EPOCH_MASK = 0x3fffull << LB_EPOCH_SHIFT;
constexpr uint64_t LB_VALUE = (1ull << LB_EPOCH_SHIFT) - 1;
constexpr uint32_t LB_EPOCHS = 1u << 14;
constexpr int64_t LB_SPIN_LIMIT = 1ll << 22;
constexpr uint64_t ERR_LOOKBACK = 16;     // bit set in the caller's error word on a spin-limit exit

// Workspace header (uint32 words at the start of the pool).
enum { H_TILE_SORT = 0, H_TILE_SCAN = RS_MAX_PASSES, H_WORDS = 64 };

// ---- look-back ------------------------------------------------------------------------

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of `agg` over tiles 0..tile-1 for one counter; the word of
// tile t for this counter is status[t * stride].  Publishes the tile's count
// first and its inclusive prefix last.  Predecessors are read LB_WINDOW at a time
// (independent loads in flight), newest first, up to the first inclusive prefix;
// a word not yet published stops the window and is read again.
constexpr int LB_WINDOW = 16;
__device__ uint64_t lookback(uint64_t *status, int64_t stride, uint32_t tile, uint64_t agg, uint64_t epoch,
                             int64_t *err) {
    if (tile == 0) {
        lb_store(&status[0], LB_PRE | epoch | agg);
        return 0;
    }
    lb_store(&status[(int64_t)tile * stride], LB_AGG | epoch | agg);
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;  // newest tile not yet accounted for
    int64_t spins = 0;
    // the direct predecessor alone first: in a long launch it has usually
    // published its inclusive prefix already
    {
        const uint64_t x = lb_load(&status[t * stride]);
        if ((x & LB_EPOCH_MASK) == epoch && (x & LB_FLAGS) != 0) {
            excl += x & LB_VALUE;
            t = (x & LB_FLAGS) == LB_PRE ? -1 : t - 1;
        }
    }
    while (t >= 0) {
        uint64_t w[LB_WINDOW];
#pragma unroll
        for (int k = 0; k < LB_WINDOW; ++k) w[k] = t - k >= 0 ? lb_load(&status[(t - k) * stride]) : 0;
        bool stop = false, done = false;
        int used = 0;
#pragma unroll
        for (int k = 0; k < LB_WINDOW; ++k) {
            if (stop || t - k < 0) {
                stop = true;
                continue;
            }
            const uint64_t x = w[k];
            if ((x & LB_EPOCH_MASK) != epoch || (x & LB_FLAGS) == 0) {
                stop = true;  // not published yet: resume at this tile
                continue;
            }
            excl += x & LB_VALUE;
            used = k + 1;
            if ((x & LB_FLAGS) == LB_PRE) {
                done = true;
                stop = true;
            }
        }
        if (done) break;
        if (used == 0) {
            if (++spins > LB_SPIN_LIMIT) {
                atomicOr((unsigned long long *)err, (unsigned long long)ERR_LOOKBACK);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        t -= used;
    }
    lb_store(&status[(int64_t)tile * stride], LB_PRE | epoch | ((excl + agg) & LB_VALUE));
    return excl;
}

// Tile id of this workgroup; the workgroup that takes the last id resets the
// counter for the next launch (every other workgroup has taken its id by then).
__device__ __forceinline__ uint32_t take_tile(uint32_t *ctr, uint32_t *s_tile) {
    if (threadIdx.x == 0) {
        const uint32_t t = atomicAdd(ctr, 1u);
        if (t == gridDim.x - 1) atomicExch(ctr, 0u);
        *s_tile = t;
    }
    __syncthreads();
    return *s_tile;
}

// Lanes of the wave whose d (8 bits) equals this lane's, among `active`.
__device__ __forceinline__ uint64_t match8(uint32_t d, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// ---- radix sort kernels -----------------------------------------------------------------

// Digit counts of every pass, added to ghist[pass][digit].
// Digit p holds key bits [8p, min(8p + 8, bits)): bits above `bits` never order.
__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift, uint32_t mask) {
    return (uint32_t)(k >> shift) & mask;
}
__host__ __device__ __forceinline__ uint32_t digit_mask(int bits, int shift) {
    const int b = bits - shift < RS_BITS ? bits - shift : RS_BITS;
    return (1u << b) - 1u;
}

// The counts alternate between two sets per sort call: this call adds into
// `ghist` (cleared by the previous call) and clears `gnext` for the next call
// (its last reader, the previous call's passes, has finished on this stream).
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                        int passes, int bits, uint32_t *ghist, uint32_t *gnext) {
    __shared__ uint32_t h[RS_WAVES][RS_MAX_PASSES][RS_RADIX];
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < RS_MAX_PASSES * RS_RADIX; i += RS_THREADS) gnext[i] = 0;
    uint32_t *hf = &h[0][0][0];
    for (int i = threadIdx.x; i < RS_WAVES * RS_MAX_PASSES * RS_RADIX; i += RS_THREADS) hf[i] = 0;
    __syncthreads();
    const int wv = threadIdx.x / WAVE;
    const int64_t stride = gstride();
    for (int64_t i = gtid(); i < n; i += stride) {
        const uint64_t k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&h[wv][p][digit_of(k, RS_BITS * p, digit_mask(bits, RS_BITS * p))], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * RS_RADIX; i += RS_THREADS) {
        uint32_t c = 0;
        for (int w = 0; w < RS_WAVES; ++w) c += (&h[w][0][0])[i];
        if (c) atomicAdd(&ghist[i], c);
    }
}

// One digit pass over tiles of THREADS * ITEMS keys.  Keys of a tile are read
// wave-striped (lane l of wave w holds key w * ITEMS * 64 + i * 64 + l of the tile
// for i < ITEMS), so ranking items in order i and, inside an item, by lane keeps
// the input order: the sort is stable.  Keys and then values are staged in LDS in
// sorted order and written out in runs of one digit (one LDS buffer for both, and
// one byte of digit per slot instead of output positions in registers).
template <int ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_pass(const uint64_t *__restrict__ kin,
                                                        const int32_t *__restrict__ vin, uint64_t *kout,
                                                        int32_t *vout, int64_t n, int shift, uint32_t dmask,
                                                        const uint32_t *__restrict__ gcount, uint64_t *status,
                                                        uint32_t *tile_ctr, uint64_t epoch, int64_t *err) {
    constexpr int TILE = RS_THREADS * ITEMS;
    __shared__ uint64_t s_stage[TILE];               // keys, then values (as 32-bit words)
    __shared__ uint8_t s_digit[TILE];                // digit of each staged slot
    __shared__ uint32_t s_wcnt[RS_WAVES][RS_RADIX];  // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_dstart[RS_RADIX];          // first slot of each digit in the tile
    __shared__ int64_t s_gstart[RS_RADIX];           // first output position of each digit's keys
    __shared__ uint32_t s_wtot[RS_WAVES];
    __shared__ uint32_t s_gtot[RS_WAVES];
    __shared__ uint32_t s_tile;
    const uint32_t tile = take_tile(tile_ctr, &s_tile);
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    for (int i = threadIdx.x; i < RS_WAVES * RS_RADIX; i += RS_THREADS) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();

    const int64_t tbase = (int64_t)tile * TILE;
    const int64_t wbase = tbase + (int64_t)wv * (ITEMS * WAVE);
    uint64_t key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t j = wbase + i * WAVE + l;
        key[i] = j < n ? kin[j] : 0;
        val[i] = j < n ? (uint32_t)vin[j] : 0;  // loaded now, in flight during the ranking
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = wbase + i * WAVE + l < n;
        const uint32_t d = digit_of(key[i], shift, dmask);
        const uint64_t m = match8(d, ballot(valid));
        const uint32_t before = (uint32_t)__popcll(m & lanemask_lt());
        // every lane of a digit group reads the running count before its first
        // lane (the group's leader) adds the group's size
        const uint32_t old = valid ? s_wcnt[wv][d] : 0;
        wave_sync();
        if (valid && before == 0) s_wcnt[wv][d] = old + (uint32_t)__popcll(m);
        wave_sync();
        rank[i] = old + before;
    }
    __syncthreads();

    // thread d: wave offsets of digit d, the tile's count of d and its global start
    const int d = threadIdx.x;
    uint32_t cnt = 0;
    {
        uint32_t c[RS_WAVES];
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) c[w] = s_wcnt[w][d];
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            s_wcnt[w][d] = cnt;
            cnt += c[w];
        }
    }
    const uint64_t excl = lookback(status + d, RS_RADIX, tile, cnt, epoch, err);
    // exclusive scans over the digits: of the tile's counts (tile-local start of
    // digit d) and of the whole input's counts (global start of digit d)
    const uint32_t gc = gcount[d];
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t gincl = wave_incl_scan(gc);
    if (l == WAVE - 1) {
        s_wtot[wv] = incl;
        s_gtot[wv] = gincl;
    }
    __syncthreads();
    uint32_t before = 0, gbefore = 0;
    for (int w = 0; w < wv; ++w) {
        before += s_wtot[w];
        gbefore += s_gtot[w];
    }
    s_dstart[d] = before + incl - cnt;
    s_gstart[d] = (int64_t)(gbefore + gincl - gc) + (int64_t)excl;
    __syncthreads();

    // rank[i] becomes the item's slot in the tile's sorted order
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (wbase + i * WAVE + l >= n) continue;
        const uint32_t dd = digit_of(key[i], shift, dmask);
        rank[i] += s_dstart[dd] + s_wcnt[wv][dd];
        s_stage[rank[i]] = key[i];
        s_digit[rank[i]] = (uint8_t)dd;
    }
    __syncthreads();
    const int tn = (int)min((int64_t)TILE, n - tbase);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int j = threadIdx.x + i * RS_THREADS;
        if (j >= tn) continue;
        const uint32_t dd = s_digit[j];
        const int64_t o = s_gstart[dd] + (j - (int64_t)s_dstart[dd]);
        if (o < 0 || o >= n) continue;  // only after a look-back spin-limit exit (error already set)
        kout[o] = s_stage[j];
    }
    __syncthreads();
    uint32_t *s_val = reinterpret_cast<uint32_t *>(s_stage);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (wbase + i * WAVE + l < n) s_val[rank[i]] = val[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int j = threadIdx.x + i * RS_THREADS;
        if (j >= tn) continue;
        const uint32_t dd = s_digit[j];
        const int64_t o = s_gstart[dd] + (j - (int64_t)s_dstart[dd]);
        if (o < 0 || o >= n) continue;
        vout[o] = (int32_t)s_val[j];
    }
}

// ---- exclusive scan of int64 ----------------------------------------------------------------

// One tile of 4,096 values per workgroup; each wave scans its 1,024 values as 16
// rows of 64 (coalesced), the waves' totals are combined in LDS and the tile's
// total goes through the look-back.
__global__ __launch_bounds__(SC_THREADS) void k_scan_excl(const int64_t *__restrict__ in, int64_t *out,
                                                          int64_t n, uint64_t *status, uint32_t *tile_ctr,
                                                          uint64_t epoch, int64_t *err) {
    __shared__ int64_t s_wtot[SC_THREADS / WAVE];
    __shared__ int64_t s_prefix;
    __shared__ uint32_t s_tile;
    const uint32_t tile = take_tile(tile_ctr, &s_tile);
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    const int64_t wbase = (int64_t)tile * SC_TILE + (int64_t)wv * (SC_ITEMS * WAVE);
    int64_t v[SC_ITEMS];
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        const int64_t j = wbase + i * WAVE + l;
        v[i] = j < n ? in[j] : 0;
    }
    int64_t carry = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        const int64_t incl = wave_incl_scan(v[i]);
        const int64_t row = __shfl(incl, WAVE - 1, WAVE);
        v[i] = carry + incl - v[i];
        carry += row;
    }
    if (l == 0) s_wtot[wv] = carry;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < SC_THREADS / WAVE; ++w) tot += s_wtot[w];
        s_prefix = (int64_t)lookback(status, 1, tile, (uint64_t)tot & LB_VALUE, epoch, err);
    }
    __syncthreads();
    int64_t base = s_prefix;
    for (int w = 0; w < wv; ++w) base += s_wtot[w];
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        const int64_t j = wbase + i * WAVE + l;
        if (j < n) out[j] = base + v[i];
    }
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// ---- host side ------------------------------------------------------------------------------

static inline int blocks_for(int64_t n, int per, int cap) {
    int64_t b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

// Pool layout (bytes): header words | ghist | gbase | status words | keys | values.
struct PoolLayout {
    size_t ghist, gbase, status, keys, vals, total;
};
static PoolLayout layout(int64_t status_words, int64_t n_keys) {
    PoolLayout L;
    L.ghist = 256;
    L.gbase = L.ghist + sizeof(uint32_t) * RS_MAX_PASSES * RS_RADIX;  // the second count set
    L.status = L.gbase + sizeof(uint32_t) * RS_MAX_PASSES * RS_RADIX;
    L.keys = L.status + sizeof(uint64_t) * (size_t)status_words;
    L.keys = (L.keys + 255) & ~(size_t)255;
    L.vals = L.keys + sizeof(uint64_t) * (size_t)n_keys;
    L.total = L.vals + sizeof(int32_t) * (size_t)n_keys + 256;
    return L;
}

// Make the pool hold `words` status words and `keys` ping-pong keys and values.  A
// new pool starts all zero (header, counts, status); status words that an existing
// pool's layout newly covers held scratch keys, so they are cleared.
static int prepare(SortWork &w, int64_t words, int64_t keys, hipStream_t s, PoolLayout *L) {
    words = std::max(words, w.status_words);
    keys = std::max(keys, w.key_cap);
    *L = layout(words, keys);
    if (!w.pool.p || w.pool.cap < L->total) {
        DG_TRY(w.pool.ensure(L->total));
        DG_TRY(fill_u64_on(reinterpret_cast<uint64_t *>(w.pool.p), 0, (int64_t)(w.pool.cap / 8), s));
        w.epoch = 0;
    } else if (words > w.status_words) {
        uint64_t *status = reinterpret_cast<uint64_t *>(w.pool.p + L->status);
        DG_TRY(fill_u64_on(status + w.status_words, 0, words - w.status_words, s));
    }
    w.status_words = words;
    w.key_cap = keys;
    return DG_OK;
}

int fill_u64_on(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DG_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

// Next look-back epoch as its bit field; clears the status words when the epochs wrap.
static int next_epoch(SortWork &w, uint64_t *status, int64_t words, hipStream_t s, uint64_t *bits) {
    if (++w.epoch >= LB_EPOCHS) {
        DG_TRY(fill_u64_on(status, 0, words, s));
        w.epoch = 1;
    }
    *bits = (uint64_t)w.epoch << LB_EPOCH_SHIFT;
    return DG_OK;
}

int scan_excl_i64(hipStream_t s, SortWork &w, const int64_t *in, int64_t *out, int64_t n, int64_t *err) {
    if (n <= 0) return DG_OK;
    const int64_t tiles = (n + SC_TILE - 1) / SC_TILE;
    if (tiles > INT32_MAX) return set_error(DG_EINVAL, "scan of more than 2^43 values");
    PoolLayout L;
    DG_TRY(prepare(w, tiles, 0, s, &L));
    uint8_t *base = w.pool.p;
    uint64_t *status = reinterpret_cast<uint64_t *>(base + L.status);
    uint64_t ep = 0;
    DG_TRY(next_epoch(w, status, w.status_words, s, &ep));
    hipLaunchKernelGGL(k_scan_excl, dim3((unsigned)tiles), dim3(SC_THREADS), 0, s, in, out, n, status,
                       reinterpret_cast<uint32_t *>(base) + H_TILE_SCAN, ep, err);
    DG_HIP(hipGetLastError());
    return DG_OK;
}

int radix_sort_pairs(hipStream_t s, SortWork &w, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                     int32_t *vout, int64_t n, int bits, int64_t *err) {
    if (n <= 0) return DG_OK;
    if (n > INT32_MAX) return set_error(DG_EINVAL, "sort of more than 2^31 keys");
    bits = std::max(1, std::min(bits, 64));
    const int passes = (bits + RS_BITS - 1) / RS_BITS;
    // larger tiles for large inputs (longer runs of one digit per write, fewer
    // look-back words); smaller tiles keep more workgroups busy on small ones
    const bool big = n >= (1 << 20);
    const int tile_keys = big ? RS_THREADS * 16 : RS_TILE;
    const int64_t tiles = (n + tile_keys - 1) / tile_keys;
    PoolLayout L;
    DG_TRY(prepare(w, tiles * RS_RADIX, n, s, &L));
    const int64_t words = w.status_words;
    uint8_t *base = w.pool.p;
    uint32_t *hdr = reinterpret_cast<uint32_t *>(base);
    uint32_t *ghist = reinterpret_cast<uint32_t *>(base + L.ghist);
    uint32_t *gbase = reinterpret_cast<uint32_t *>(base + L.gbase);
    uint64_t *status = reinterpret_cast<uint64_t *>(base + L.status);
    uint64_t *tk = reinterpret_cast<uint64_t *>(base + L.keys);
    int32_t *tv = reinterpret_cast<int32_t *>(base + L.vals);
    uint32_t *gcur = (w.calls & 1) ? gbase : ghist, *gnext = (w.calls & 1) ? ghist : gbase;
    ++w.calls;
    hipLaunchKernelGGL(k_rs_hist, dim3(blocks_for(n, RS_THREADS * 4, 2048)), dim3(RS_THREADS), 0, s, kin, n,
                       passes, bits, gcur, gnext);
    DG_HIP(hipGetLastError());
    // ping-pong so that the last pass writes kout/vout: odd pass counts start there
    const uint64_t *ki = kin;
    const int32_t *vi = vin;
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint64_t *ko = to_out ? kout : tk;
        int32_t *vo = to_out ? vout : tv;
        uint64_t ep = 0;
        DG_TRY(next_epoch(w, status, words, s, &ep));
        hipLaunchKernelGGL(big ? k_rs_pass<16> : k_rs_pass<RS_ITEMS>, dim3((unsigned)tiles), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n, RS_BITS * p,
                           digit_mask(bits, RS_BITS * p), gcur + p * RS_RADIX, status, hdr + H_TILE_SORT + p, ep, err);
        DG_HIP(hipGetLastError());
        ki = ko;
        vi = vo;
    }
    return DG_OK;
}

}  // namespace dg
