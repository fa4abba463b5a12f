/* Fast core of the seeded R-MAT generator (same stream as the numpy definition
 * in graphgen/__init__.py): candidate drawing and first-occurrence dedup.
 * Holds no arithmetic of the dynamic-graph method. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Candidate i (start <= i < start+count): word j is draw number i*words + j of
 * the stream; each level consumes a 16-bit slice, low slice first. */
void gg_rmat_candidates(uint64_t seed, int scale, int64_t start, int64_t count,
                        uint32_t ta, uint32_t tab, uint32_t tabc,
                        int64_t *src, int64_t *dst) {
    const int words = (scale + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < count; ++c) {
        uint64_t i = (uint64_t)(start + c);
        int64_t s = 0, d = 0;
        int level = 0;
        for (int j = 0; j < words; ++j) {
            uint64_t w = mix64(seed + (i * (uint64_t)words + (uint64_t)(j + 1)) * GOLDEN);
            for (int q = 0; q < 4 && level < scale; ++q, ++level) {
                uint32_t r = (uint32_t)((w >> (16 * q)) & 0xFFFFu);
                int sb = r >= tab;
                int db = (r >= ta && r < tab) || r >= tabc;
                s = (s << 1) | sb;
                d = (d << 1) | db;
            }
        }
        src[c] = s;
        dst[c] = d;
    }
}

/* LSD radix sort of (key, index) pairs on the low key_bits bits, 11 bits a pass. */
static void radix_pairs(uint64_t *k, uint32_t *v, int64_t n, int key_bits,
                        uint64_t *tk, uint32_t *tv) {
    const int B = 11, R = 1 << B;
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * R);
    for (int sh = 0; sh < key_bits; sh += B) {
        memset(cnt, 0, sizeof(int64_t) * R);
        for (int64_t i = 0; i < n; ++i) cnt[(k[i] >> sh) & (R - 1)]++;
        int64_t acc = 0;
        for (int r = 0; r < R; ++r) { int64_t c = cnt[r]; cnt[r] = acc; acc += c; }
        for (int64_t i = 0; i < n; ++i) {
            int64_t p = cnt[(k[i] >> sh) & (R - 1)]++;
            tk[p] = k[i];
            tv[p] = v[i];
        }
        uint64_t *x = k; k = tk; tk = x;
        uint32_t *y = v; v = tv; tv = y;
        /* swap back so the caller's arrays hold the result after an even number of
         * passes; handled below by copying when the pass count is odd */
    }
    int passes = (key_bits + B - 1) / B;
    if (passes & 1) {
        memcpy(tk, k, sizeof(uint64_t) * n);
        memcpy(tv, v, sizeof(uint32_t) * n);
    }
    free(cnt);
}

/* Indices (ascending) of the first occurrence of every distinct key, truncated to
 * ``want``.  Returns the number written to out_idx. */
int64_t gg_first_unique(const uint64_t *keys, int64_t n, int key_bits, int64_t want,
                        int64_t *out_idx) {
    uint64_t *k = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *tk = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint32_t *v = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *tv = (uint32_t *)malloc(sizeof(uint32_t) * n);
    unsigned char *first = (unsigned char *)calloc((size_t)n, 1);
    memcpy(k, keys, sizeof(uint64_t) * n);
    for (int64_t i = 0; i < n; ++i) v[i] = (uint32_t)i;
    radix_pairs(k, v, n, key_bits, tk, tv);
    /* stable sort: within a run of equal keys the smallest index comes first */
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || k[i] != k[i - 1]) first[v[i]] = 1;
    int64_t c = 0;
    for (int64_t i = 0; i < n && c < want; ++i)
        if (first[i]) out_idx[c++] = i;
    free(k); free(tk); free(v); free(tv); free(first);
    return c;
}
