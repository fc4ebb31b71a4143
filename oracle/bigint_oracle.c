/*
 * CPU oracle for batched big-integer addition and multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library and is deliberately plain and slow: it is the definition of
 * the results, written out, not an implementation of the paper's parallel
 * algorithms (scan-based carry propagation, load-balanced convolution, NTT),
 * which all reach exactly the same results.
 *
 * Representation (Section 2): an integer is an array of M little-endian limbs
 * in base x = 2^32, a = a_0 + a_1 x + ... + a_{M-1} x^{M-1}.  Integers with
 * 64-bit limbs are handled by the caller as twice as many 32-bit limbs, which
 * is the same byte string on a little-endian host.
 *
 * Batches are instance-major and contiguous: pair p occupies limbs
 * [p*n, (p+1)*n) of each input.  Pairs are independent; the batch loops run
 * one pair per OpenMP task, which changes nothing in the per-pair arithmetic.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <omp.h>

/* Section 2, the sequential procedure of Fig. 1 (left): add corresponding
 * limbs together with the previous carry in a type of double width; the
 * result limb is the remainder and the next carry the quotient of the sum by
 * the base.  Returns the carry out of the top limb. */
static uint32_t add_one(const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n) {
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
        uint64_t s = (uint64_t)a[i] + (uint64_t)b[i] + carry;
        out[i] = (uint32_t)s;
        carry = s >> 32;
    }
    return (uint32_t)carry;
}

/* Eq. (1), Section 3.1: C_k = sum_{i+j=k} A_i B_j, here for the full product
 * (k = 0 .. 2n-1, no truncation to n limbs).  Schoolbook rows: for each limb
 * a_i, add a_i * b shifted by i limbs into the result, propagating the carry
 * along the row.  Every intermediate fits in 64 bits:
 * (2^32-1)^2 + 2 (2^32-1) = 2^64 - 1. */
static void mul_one(const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n) {
    memset(out, 0, 2 * n * sizeof(uint32_t));
    for (size_t i = 0; i < n; ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < n; ++j) {
            uint64_t t = (uint64_t)a[i] * (uint64_t)b[j] + (uint64_t)out[i + j] + carry;
            out[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        out[i + n] = (uint32_t)carry;
    }
}

static int pick_threads(int threads) {
    return threads > 0 ? threads : omp_get_max_threads();
}

/* Batched addition: out[p] = (a[p] + b[p]) mod 2^(32n); carry[p] = the carry
 * out of the top limb (carry may be NULL).  Returns the thread count used. */
int oracle_add(const uint32_t *a, const uint32_t *b, uint32_t *out, uint8_t *carry,
               uint64_t n, uint64_t batch, int threads) {
    int t = pick_threads(threads);
    #pragma omp parallel for num_threads(t) schedule(dynamic, 64)
    for (int64_t p = 0; p < (int64_t)batch; ++p) {
        uint32_t c = add_one(a + p * n, b + p * n, out + p * n, n);
        if (carry) carry[p] = (uint8_t)c;
    }
    return t;
}

/* Batched full product: out[p] (2n limbs) = a[p] * b[p]. */
int oracle_mul(const uint32_t *a, const uint32_t *b, uint32_t *out,
               uint64_t n, uint64_t batch, int threads) {
    int t = pick_threads(threads);
    #pragma omp parallel for num_threads(t) schedule(dynamic, 1)
    for (int64_t p = 0; p < (int64_t)batch; ++p)
        mul_one(a + p * n, b + p * n, out + 2 * p * n, n);
    return t;
}

/* Ragged batch: pair p has n[p] limbs at a + a_off[p], b + b_off[p]; its
 * product (2 n[p] limbs) goes to out + out_off[p].  Offsets are in limbs. */
int oracle_mul_ragged(const uint32_t *a, const uint32_t *b, uint32_t *out,
                      const uint64_t *a_off, const uint64_t *b_off, const uint64_t *out_off,
                      const uint32_t *n, uint64_t count, int threads) {
    int t = pick_threads(threads);
    #pragma omp parallel for num_threads(t) schedule(dynamic, 1)
    for (int64_t p = 0; p < (int64_t)count; ++p)
        mul_one(a + a_off[p], b + b_off[p], out + out_off[p], n[p]);
    return t;
}

/* Ragged batch addition, same conventions (out has n[p] limbs). */
int oracle_add_ragged(const uint32_t *a, const uint32_t *b, uint32_t *out, uint8_t *carry,
                      const uint64_t *a_off, const uint64_t *b_off, const uint64_t *out_off,
                      const uint32_t *n, uint64_t count, int threads) {
    int t = pick_threads(threads);
    #pragma omp parallel for num_threads(t) schedule(dynamic, 16)
    for (int64_t p = 0; p < (int64_t)count; ++p) {
        uint32_t c = add_one(a + a_off[p], b + b_off[p], out + out_off[p], n[p]);
        if (carry) carry[p] = (uint8_t)c;
    }
    return t;
}
