/*
 * Seeded, counter-based input generator shared by the oracle tests and the
 * HIP path tests/benchmark.  It holds no big-integer arithmetic: it only
 * produces pseudo-random 64-bit words.
 *
 * Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used as a counter-based hash:
 *
 *   key(seed, cfg, pair, operand) = sm(sm(seed ^ sm(cfg)) ^ (2*pair + operand))
 *   word(key, j)                  = sm(key + j * 0xD1B54A32D192ED03)
 *
 * where sm(x) is the SplitMix64 output function applied to x + golden gamma.
 * All arithmetic wraps modulo 2^64.  The Python reference definition in
 * workloads/__init__.py computes the same words for small cases.
 */
#include <stdint.h>
#include <stddef.h>

static inline uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t wl_key(uint64_t seed, uint64_t cfg, uint64_t pair, uint64_t operand) {
    return sm64(sm64(seed ^ sm64(cfg)) ^ (2 * pair + operand));
}

uint64_t wl_hash(uint64_t x) { return sm64(x); }

/* Fill out[p * words + j] = word(key(seed, cfg, pairs[p], operand), j)
 * for p < npairs, j < words.  `pairs` may be NULL, meaning pairs[p] = pair0 + p. */
void wl_fill(uint64_t seed, uint64_t cfg, uint64_t pair0, const uint64_t *pairs,
             uint64_t npairs, uint64_t operand, uint64_t words, uint64_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)npairs; ++p) {
        uint64_t pair = pairs ? pairs[p] : pair0 + (uint64_t)p;
        uint64_t key = wl_key(seed, cfg, pair, operand);
        uint64_t *dst = out + (uint64_t)p * words;
        for (uint64_t j = 0; j < words; ++j)
            dst[j] = sm64(key + j * 0xD1B54A32D192ED03ull);
    }
}

/* Ragged fill: pair p (index pairs[p]) gets nwords[p] words at out + offsets[p]. */
void wl_fill_ragged(uint64_t seed, uint64_t cfg, const uint64_t *pairs, uint64_t npairs, uint64_t operand,
                    const uint64_t *nwords, const uint64_t *offsets, uint64_t *out) {
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < (int64_t)npairs; ++p) {
        uint64_t key = wl_key(seed, cfg, pairs[p], operand);
        uint64_t *dst = out + offsets[p];
        for (uint64_t j = 0; j < nwords[p]; ++j)
            dst[j] = sm64(key + j * 0xD1B54A32D192ED03ull);
    }
}
