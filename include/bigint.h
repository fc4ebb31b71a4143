/*
 * bigint.h -- C ABI of the MI355X (gfx950) batched big-integer library.
 *
 * Method: Oancea & Watt, "GPU Implementations for Midsize Integer Addition
 * and Multiplication" (arXiv 2405.14642).  One integer (or a few small ones)
 * per wavefront/workgroup, operands held in VGPRs and LDS.
 *
 * Representation (Section 2): an integer of n limbs of w bits is the
 * little-endian limb array a_0 .. a_{n-1}, value sum a_i 2^(w i).  A batch is
 * instance-major and contiguous: instance p occupies limbs [p n, (p+1) n).
 * w is 32 or 64 per call; n * w may not exceed BI_MAX_BITS.
 *
 * Memory and ownership: every data pointer is a device pointer (HBM) owned by
 * the caller, who must keep it alive until the work queued on `stream` has
 * completed.  Pointers must be aligned to the limb size.  The library never
 * frees or retains them.  A context owns only its own tables and scratch.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Every compute
 * entry point only validates and enqueues; results are ready once the stream
 * has been synchronised.
 *
 * Errors: return codes only; nothing aborts and no C++ exception crosses the
 * ABI.  Argument validation is synchronous, touches no GPU state, runs before
 * any HIP call and leaves outputs untouched when it fails.  Launch failures
 * are reported as BI_EHIP; asynchronous device faults surface at the caller's
 * next synchronisation.  bi_last_error() gives a message for the last failing
 * call on the calling host thread.  A context is not thread-safe: use one per
 * host thread or serialise calls.  bigmul (NTT and large-product MFMA paths),
 * bigmul_v and bigadd_large use one scratch buffer owned by the context: such
 * calls on different streams of one context must not overlap in time (order
 * them with events, or use a context per stream).  When a call needs more
 * scratch than the context holds, it synchronises the device and reallocates.
 */
#ifndef BIGINT_MI355X_H
#define BIGINT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BI_MAX_BITS (1u << 18) /* largest integer, in bits (Section 1: up to ~2^18 bits) */
#define BI_MAX_LARGE_BITS (1ull << 40) /* largest single integer of bigadd_large, in bits */
#define BI_MAX_LARGE_MUL_BITS (1u << 24) /* largest operand of bigmul_large, in bits */

typedef enum bi_status {
    BI_OK = 0,
    BI_EINVAL = -1, /* null pointer, null context, zero size, unknown option  */
    BI_ESIZE = -2,  /* n_limbs * limb_bits > BI_MAX_BITS, or batch too large  */
    BI_ELIMB = -3,  /* limb_bits not 32 or 64, or a pointer not limb-aligned  */
    BI_EALIAS = -4, /* output overlaps an input where the operation forbids it */
    BI_EHIP = -5,   /* a HIP runtime call or kernel launch failed             */
    BI_ENOMEM = -6, /* device allocation of context scratch failed            */
    BI_EALGO = -7,  /* the requested multiplication algorithm cannot run this size */
    BI_ENODEV = -8  /* no usable gfx950 device                                 */
} bi_status;

typedef enum bi_mul_algo {
    BI_MUL_AUTO = 0,         /* the context's tuned choice for (n, batch)            */
    BI_MUL_SCHOOL_VALU = 1,  /* load-balanced schoolbook on the VALU (Section 3)     */
    BI_MUL_SCHOOL_MFMA = 2,  /* schoolbook on int8 MFMA, signed 8-bit digits         */
    BI_MUL_NTT = 3,          /* NTT over two word-size primes + CRT (Section 4)       */
    BI_MUL_NTT_PF64 = 4,     /* NTT over the one 64-bit prime PrimeField64 (Section 4.1) */
    BI_MUL_KARATSUBA = 5     /* Karatsuba levels over a batched base product (sizes by  */
                             /* choice of algorithm, left open in Section 1)           */
} bi_mul_algo;

typedef struct bi_ctx bi_ctx;

/* Create a context on HIP device `device` (the device is made current for
 * the call).  Allocates the context's device tables (NTT twiddles).
 * Returns BI_ENODEV if the device does not exist or is not gfx950,
 * BI_ENOMEM / BI_EHIP on allocation or copy failure; *out is NULL then. */
bi_status bi_ctx_create(int device, bi_ctx **out);

/* Release a context and its device tables.  Waits for nothing: the caller
 * must have synchronised every stream that used it.  NULL is ignored. */
void bi_ctx_destroy(bi_ctx *ctx);

/* Static description of a status code.  Never NULL. */
const char *bi_status_str(int status);

/* Message for the last failing call on this host thread ("" if none). */
const char *bi_last_error(void);

/*
 * bigadd -- Section 2 (addition as a carry-propagation scan, Fig. 2) and its
 * batched form bbadd.  For each of `batch` instances:
 *     out[p]       = (a[p] + b[p]) mod 2^(n_limbs * limb_bits)
 *     carry_out[p] = floor((a[p] + b[p]) / 2^(n_limbs * limb_bits))  (0 or 1)
 * a, b, out: batch * n_limbs limbs each.  carry_out: batch bytes, or NULL.
 * out may be identical to a or to b (in-place); any other overlap of out or
 * carry_out with the inputs is BI_EALIAS.
 */
bi_status bigadd(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out,
                 uint32_t n_limbs, uint32_t limb_bits, uint64_t batch, void *stream);

/*
 * bigadd_large -- Section 2's addition (a carry-propagation scan) for ONE
 * integer of any length, carried across workgroups; the paper's kernels stop
 * at one block and leave longer integers to slower fall-back versions
 * (Section 5.1).  Computes
 *     out        = (a + b) mod 2^(n_limbs * limb_bits)
 *     *carry_out = floor((a + b) / 2^(n_limbs * limb_bits))  (0 or 1)
 * a, b, out: n_limbs limbs of limb_bits (32 or 64) bits each, little-endian,
 * device memory owned by the caller; 1 <= n_limbs and n_limbs * limb_bits <=
 * BI_MAX_LARGE_BITS (BI_EINVAL / BI_ESIZE), and device memory bounds it
 * further.  carry_out: one device byte, or NULL.  out may be identical to a or
 * to b (in-place); any other overlap of out or carry_out with the inputs is
 * BI_EALIAS.  Pointers must be limb-aligned (BI_ELIMB); 16-byte alignment of
 * a, b and out gives the widest accesses.  Runs four kernels on `stream`
 * (tile sums with tile carry summaries, a scan of the summaries, carry
 * fix-up, a walk of tiles the carry crosses), or up to 512 tiles two (the
 * summaries, then each tile's sum with its carry-in found from the summaries
 * below it), using about 6 bytes of context scratch per tile of 1024
 * chunks; BI_ENOMEM if that scratch cannot grow.
 * Asynchronous like every call.
 */
bi_status bigadd_large(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out,
                       uint64_t n_limbs, uint32_t limb_bits, void *stream);

/*
 * bigmul_large -- the full product (eq. (1) of Section 3.1) of ONE pair of
 * integers beyond the batched kernels' 2^18 bits, the paper's slower
 * fall-back sizes (Section 5.1):  out (2 n_limbs limbs) = a * b.
 * a, b: n_limbs limbs of limb_bits (32 or 64) bits; 1 <= n_limbs and
 * n_limbs * limb_bits <= BI_MAX_LARGE_MUL_BITS (BI_EINVAL / BI_ESIZE);
 * out must not overlap a or b (BI_EALIAS); pointers limb-aligned (BI_ELIMB).
 * algo BI_MUL_AUTO or BI_MUL_NTT: a two-dimensional NTT convolution (n log n
 * work): the operands are cut into k <= 64 blocks of block_bits bits (a
 * power of two in [2^14, 2^18]; 0 lets the library choose: the smallest of at
 * least 2^16 bits that gives at most 32 blocks, or 2^18), each block's 16-bit
 * coefficients are transformed along the block (length 4 * block words)
 * and the results across the blocks (length 2k rounded up to a power of
 * two), modulo the two primes of BI_MUL_NTT; pointwise products, both
 * inverses, CRT, a fold into low and high words (with the carry status of
 * every 2048-word tile) and one addition kernel give the product.  Scratch:
 * 16 k (4 block words) bytes of transforms plus about 16 n bytes of low and
 * high words (n = 32-bit words of an operand).
 * algo BI_MUL_SCHOOL_VALU, BI_MUL_SCHOOL_MFMA, BI_MUL_NTT_PF64 or
 * BI_MUL_KARATSUBA: k^2 block products of that algorithm (block_bits 2^16,
 * 2^17 or 2^18, 0: 2^16 up to 2^20-bit operands, 2^18 above) as one ragged
 * batch, a column-sum kernel and bigadd_large's kernels; scratch about
 * 8 k^2 (block words) bytes of block products plus the batch's own.
 * BI_EALGO if the algorithm cannot run the block size; BI_EINVAL for an
 * unknown algorithm or block size.  BI_ENOMEM if the context's scratch
 * cannot grow.  Asynchronous like every call.
 */
/* The block size (bits) and block count bigmul_large picks for block_bits = 0
 * (host only; errors as bigmul_large's size and algorithm checks). */
bi_status bi_mul_large_plan(uint64_t n_limbs, uint32_t limb_bits, int algo, uint32_t *block_bits, uint32_t *blocks);

bi_status bigmul_large(bi_ctx *ctx, const void *a, const void *b, void *out, uint64_t n_limbs, uint32_t limb_bits,
                       int algo, uint32_t block_bits, void *stream);

/*
 * bigmul -- full product, eq. (1) of Section 3.1 without truncation: for each
 * instance out[p] (2 * n_limbs limbs) = a[p] * b[p].  The paper's same-length
 * product (Figs. 4-6) is the low n_limbs limbs of out[p].
 * a, b: batch * n_limbs limbs; out: batch * 2 * n_limbs limbs, which must not
 * overlap a or b (BI_EALIAS).  algo selects the method:
 *   BI_MUL_SCHOOL_VALU   Section 3: each thread owns load-balanced output
 *                        coefficients, accumulating double-width products and
 *                        an overflow count; then a carry scan (Section 2).
 *   BI_MUL_SCHOOL_MFMA   the same convolution on int8 matrix cores, over
 *                        balanced signed base-256 digits with int32 sums that
 *                        cannot overflow, then a signed carry normalisation.
 *   BI_MUL_NTT           Section 4: number-theoretic transforms modulo primes
 *                        k 2^m + 1 over 16-bit coefficients, recombined by the
 *                        Chinese remainder theorem, then a carry scan.
 *   BI_MUL_NTT_PF64      Section 4.1's PrimeField64, p = 29 2^57 + 1: one
 *                        prime above every coefficient bound (2^46), 64-bit
 *                        Montgomery arithmetic; the product is taken as its
 *                        cyclic and negacyclic halves (transforms of half the
 *                        padded length), recombined, then a carry scan.
 *   BI_MUL_KARATSUBA     levels of the subtractive Karatsuba split (a0 b0,
 *                        a1 b1 and |a0 - a1| |b0 - b1| for halves a0, a1,
 *                        b0, b1) until the operands have at most 1024 words
 *                        (2^15 bits), whose products run as one batch with
 *                        the tuned algorithm of that size; 3^levels base
 *                        products per pair instead of 4^levels.
 *   BI_MUL_AUTO          the tuned choice of the above for the size class.
 * Results are exact (bit-identical across algorithms).
 */
bi_status bigmul(bi_ctx *ctx, const void *a, const void *b, void *out,
                 uint32_t n_limbs, uint32_t limb_bits, uint64_t batch, int algo, void *stream);

/*
 * bigmul_noalloc -- bigmul for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same products, bit-identical, with every scratch buffer
 * the kernels use (NTT transforms, the large-product MFMA slots, Karatsuba
 * levels) in one fixed device array of BI_NOALLOC_SCRATCH_BYTES per GPU that
 * is part of the library's code object and is held until the process ends.
 * The call makes no device allocation or free.  Batches whose scratch
 * exceeds the array run in rounds that fit it; BI_ESIZE if a single product
 * needs more (never at n_limbs * limb_bits <= BI_MAX_BITS).  Arguments,
 * errors and aliasing rules are bigmul's.  Every call on one GPU, from any
 * context, stream or host thread, uses that GPU's one array and leaves its
 * contents behind: calls that overlap in time on one GPU race and must be
 * ordered by the caller (one stream, or events).
 */
#define BI_NOALLOC_SCRATCH_BYTES (64u << 20)

bi_status bigmul_noalloc(bi_ctx *ctx, const void *a, const void *b, void *out, uint32_t n_limbs,
                         uint32_t limb_bits, uint64_t batch, int algo, void *stream);

/*
 * bi_mul_plan -- what bigmul runs for n_limbs-limb operands with `algo` on
 * this context (host only, no HIP call): the algorithm (BI_MUL_AUTO resolved
 * through the tuning table), and for BI_MUL_KARATSUBA the number of levels,
 * the words of each base product and the base products' algorithm (without
 * Karatsuba: 0 levels, n_limbs * limb_bits / 32 words, the algorithm itself).
 * Errors as bigmul's argument checks (BI_ELIMB, BI_EINVAL, BI_ESIZE), and
 * BI_EALGO if the algorithm cannot run that size.
 */
typedef struct bi_mul_plan_info {
    int algo;
    int kara_levels;
    uint32_t base_limbs; /* 32-bit words */
    int base_algo;
} bi_mul_plan_info;

bi_status bi_mul_plan(const bi_ctx *ctx, uint32_t n_limbs, uint32_t limb_bits, int algo, bi_mul_plan_info *out);

/*
 * bi_fused -- the paper's fused programs (Section 6.1): several same-length
 * operations per instance in one kernel, each instance in one workgroup with
 * its intermediates in LDS (operands read once, the result written once).
 * All arithmetic is mod 2^(n_limbs * limb_bits), as the paper's add and its
 * same-length product (the low n limbs of eq. (1)):
 *   BI_PROG_ADD6  six additions in a chain, a + b, then + a, + b, + a, + b,
 *                 + a: out = 4 a + 3 b.
 *   BI_PROG_POLY  out = (a a + b) (b b + b) + a b (four products, three
 *                 additions).
 *   BI_PROG_MUL_LOW  out = a b: the paper's same-length product (Section 3,
 *                 Figs. 4-5), the low n limbs of eq. (1), computing only the
 *                 coefficients below n (about half the work of bigmul).
 * a, b, out: batch * n_limbs limbs; out must not overlap a or b (BI_EALIAS).
 * Unknown program: BI_EINVAL; n_limbs * limb_bits > BI_MAX_BITS: BI_ESIZE.
 */
typedef enum bi_program {
    BI_PROG_ADD6 = 1,
    BI_PROG_POLY = 2,
    BI_PROG_MUL_LOW = 3
} bi_program;

bi_status bi_fused(bi_ctx *ctx, int program, const void *a, const void *b, void *out, uint32_t n_limbs,
                   uint32_t limb_bits, uint64_t batch, void *stream);

/*
 * Ragged batches: instance p has desc[p].n_limbs limbs (>= 1) starting at limb
 * offset desc[p].a_off in a and desc[p].b_off in b; its result starts at limb
 * offset desc[p].out_off in out (n_limbs limbs for bigadd_v, 2 n_limbs for
 * bigmul_v) and its carry (bigadd_v) at carry_out[p].  `desc` is a DEVICE
 * array of `count` descriptors; its contents are not validated on the host
 * (offsets must stay inside the caller's buffers).  Output ranges of different
 * instances must not overlap each other or any input range.
 * Batching across sizes is the library's own extension (the paper's batches
 * are uniform, Section 6.1).
 */
typedef struct bi_desc {
    uint64_t a_off, b_off, out_off; /* in limbs */
    uint32_t n_limbs;
    uint32_t reserved;              /* must be 0 */
} bi_desc;

bi_status bigadd_v(bi_ctx *ctx, const void *a, const void *b, void *out, uint8_t *carry_out,
                   const bi_desc *desc, uint64_t count, uint32_t limb_bits, void *stream);

bi_status bigmul_v(bi_ctx *ctx, const void *a, const void *b, void *out,
                   const bi_desc *desc, uint64_t count, uint32_t limb_bits, int algo, void *stream);

/*
 * Tuning.  BI_MUL_AUTO picks a multiplication algorithm per size class:
 * class k holds instances of (16 << (k-1), 16 << k] 32-bit limbs (class 0:
 * up to 16), k < BI_NUM_CLASSES.  Uniform batches (bigmul) use one table,
 * ragged batches (bigmul_v, the stream queue) another.  bi_autotune first
 * picks, per class, the VALU schoolbook's schedule (Q = 2 or 4 output words
 * per lane -- the paper's sequentialisation factor, Section 3 -- and 1..16
 * waves per workgroup), then times every algorithm (Karatsuba at each base
 * size) on synthetic operands of each class's largest size and keeps the
 * fastest for the uniform table, then times every algorithm on a ragged
 * batch of the class (sizes spread over the class) for the ragged table,
 * and the addition schedules for 2-, 4- and 8-row instances; it copies the
 * uniform per-class choice to algo_out[0 .. n_out) if not NULL.  It allocates
 * and frees about 64 MiB of device memory, may grow the context's scratch,
 * and synchronises `stream`.  bi_tune_get / bi_tune_set read or replace the
 * uniform per-class choice (BI_EALGO if an algorithm cannot run a class's
 * sizes; nothing is changed then).  Until tuned, a context uses built-in
 * tables (the choices bi_autotune made on an MI355X).
 *
 * bi_tune_save writes the context's tables (uniform and ragged algorithm,
 * VALU schedule and Karatsuba base per class, the addition schedules) to the
 * text file `path`, keyed by the
 * device's architecture name and the HIP runtime version; bi_tune_load reads
 * such a file into the context.  A file written for another architecture or
 * runtime version, a malformed one, or one naming an algorithm or schedule a
 * class cannot run is refused (BI_EINVAL, nothing changed).  Host file I/O
 * only, no HIP call; BI_EINVAL if the file cannot be opened.
 */
#define BI_NUM_CLASSES 10

bi_status bi_autotune(bi_ctx *ctx, void *stream, int *algo_out, uint32_t n_out);
bi_status bi_tune_get(const bi_ctx *ctx, int *algo_out, uint32_t n_out);
bi_status bi_tune_set(bi_ctx *ctx, const int *algo_in, uint32_t n_in);
bi_status bi_tune_save(const bi_ctx *ctx, const char *path);
bi_status bi_tune_load(bi_ctx *ctx, const char *path);
/* The VALU schoolbook schedule per class: q_out[k], waves_out[k] ((0, 0):
 * the built-in size rule applies).  Either array may be NULL.
 * bi_tune_set_valu replaces entries 0 .. n_in-1: (0, 0) restores the size
 * rule; otherwise q must be 2 or 4, waves 1, 2, 4, 8 or 16, and the schedule's
 * LDS must fit one CU for the class's largest size (BI_EINVAL otherwise;
 * nothing is changed then). */
bi_status bi_tune_get_valu(const bi_ctx *ctx, int *q_out, int *waves_out, uint32_t n_out);
bi_status bi_tune_set_valu(bi_ctx *ctx, const int *q_in, const int *waves_in, uint32_t n_in);

/* The ragged-batch table: bigmul_v and the stream queue with BI_MUL_AUTO run
 * class k's instances (spread over the class's sizes) with list_algo[k];
 * bi_autotune times every algorithm on such a batch per class.  Set / get as
 * bi_tune_set / bi_tune_get (BI_EALGO, nothing changed, if an algorithm
 * cannot run a class). */
bi_status bi_tune_get_list(const bi_ctx *ctx, int *algo_out, uint32_t n_out);
bi_status bi_tune_set_list(bi_ctx *ctx, const int *algo_in, uint32_t n_in);

/* The Karatsuba base per class: BI_MUL_KARATSUBA on class k's sizes splits
 * until the operands have at most base[k] 32-bit words (512, 1024 or 2048;
 * default 1024); bi_autotune picks it per class.  bi_tune_set_kara replaces
 * entries 0 .. n_in-1 (BI_EINVAL, nothing changed, for any other value). */
bi_status bi_tune_get_kara(const bi_ctx *ctx, uint32_t *base_out, uint32_t n_out);
bi_status bi_tune_set_kara(bi_ctx *ctx, const uint32_t *base_in, uint32_t n_in);

/*
 * Stream mode: a queue of ragged multiplication bursts over caller-owned
 * operand buffers a (a_limbs limbs), b (b_limbs) and out (out_limbs), all of
 * `limb_bits`-bit limbs.  Bursts run on the queue's own two streams (burst t
 * on the (t mod 2)-th), so consecutive bursts may overlap on the GPU; each
 * starts once its descriptors have been copied.  The queue starts after the
 * work queued on `stream` when it is opened, and `stream` waits for every
 * burst in submission order, so work queued on `stream` after a submission
 * sees that burst's results.  The caller must not change operand data, or
 * give two bursts that may be in flight overlapping output ranges, without
 * waiting for the earlier ticket.
 *
 * bi_stream_open allocates a few staging slots (each a pinned host buffer and
 * a device buffer of max_descs descriptors and class-list entries), the
 * binning and transform scratch and a side stream for the descriptor copies.
 * With use_graph == 0 every submission is binned into size classes on the
 * host and only the classes present are launched, grids sized to their
 * counts.  With use_graph != 0 it captures, for each slot, the launch
 * sequence of one burst --
 * device-side binning into size classes, then one persistent list kernel per
 * class that reads its instance count on the device -- into a HIP graph that
 * every submission replays.  The per-class algorithm is `algo`, or for
 * BI_MUL_AUTO the context's ragged-batch table at open time.  The queue keeps
 * pointers to ctx and the buffers; they must outlive it.  BI_ENOMEM / BI_EHIP
 * on allocation or capture failure (nothing is left allocated then).
 *
 * bi_stream_submit copies `count` (1 .. max_descs) HOST descriptors through a
 * slot to the device (on the side stream, ordered before the burst) and
 * enqueues the burst on `stream`; it validates every
 * descriptor first (1 <= n_limbs, n_limbs * limb_bits <= BI_MAX_BITS,
 * reserved == 0, input ranges inside a and b, output range inside out;
 * BI_EINVAL / BI_ESIZE and nothing enqueued otherwise).  It blocks only when
 * all staging slots are still in flight.  *ticket receives the burst's
 * sequence number.  bi_stream_poll sets *done to 1 once that burst's results
 * are in `out` (0 while it runs); bi_stream_wait blocks until then.
 * bi_stream_close waits for every burst and frees the queue.  A queue is not
 * thread-safe.  Descriptor semantics are those of bigmul_v.  This replaces the
 * paper's fixed-size batches (Section 6.1) by a stream of mixed sizes.
 */
typedef struct bi_stream bi_stream;

bi_status bi_stream_open(bi_ctx *ctx, const void *a, uint64_t a_limbs, const void *b, uint64_t b_limbs,
                         void *out, uint64_t out_limbs, uint32_t limb_bits, uint64_t max_descs, int algo,
                         int use_graph, void *stream, bi_stream **q);
bi_status bi_stream_submit(bi_stream *q, const bi_desc *host_descs, uint64_t count, uint64_t *ticket);
bi_status bi_stream_poll(bi_stream *q, uint64_t ticket, int *done);
bi_status bi_stream_wait(bi_stream *q, uint64_t ticket);
bi_status bi_stream_close(bi_stream *q);

/*
 * bi_ntt_field -- host-only helper for the prime-field construction of
 * Section 4.1: for an odd prime p = k 2^n + 1 (p < 2^63), returns k, the
 * two-adicity n, and the first a = 2, 3, ... for which g = a^k is a primitive
 * 2^n-th root of unity (g^(2^(n-1)) != 1), which is how the library derives
 * the roots of its NTT primes.  Makes no HIP call.  BI_EINVAL if p is not an
 * odd prime below 2^63 or out is NULL.
 */
typedef struct bi_ntt_field_info {
    uint64_t p, k;
    uint32_t two_adicity, reserved;
    uint64_t a, g;
} bi_ntt_field_info;

bi_status bi_ntt_field(uint64_t p, bi_ntt_field_info *out);

#ifdef __cplusplus
}
#endif

#endif /* BIGINT_MI355X_H */
