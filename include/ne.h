/*
 * libne -- numerical entanglement of integer streams on MI355X (gfx950).
 *
 * Implements the method of M. A. Anam and Y. Andreopoulos, "Failure
 * Mitigation in Linear, Sesquilinear and Bijective Operations On Integer
 * Data Streams Via Numerical Entanglement", IOLTS 2015:
 *
 *   1. entangle  (Sec. III, eq. (6), (14)-(15)): M >= 3 integer input streams
 *      c_m are superimposed pairwise into M entangled streams
 *          eps_m = c_m + S_l{c_{(m-1) mod M}}
 *      held in 64-bit words (w = 64), or in the paper's practical 32-bit
 *      words (w = 32: the ne_*32 calls and ne_group.word_bits);
 *   2. lsb_apply (eq. (2), (9)): one linear, sesquilinear or bijective
 *      operation runs on every entangled stream independently,
 *          delta_m = eps_m op g;
 *   3. extract_recover (eq. (10), (16)-(19)): every output d_m = c_m op g is
 *      recovered from any M-1 of the delta_m with additions and arithmetic
 *      shifts, so the loss of any single stream (fail-stop) is harmless.
 *
 * Plus the checksum method the paper compares against (Sec. II-A,
 * eq. (3)-(5)) and failure-intolerant ("plain") operations, and a batched
 * executor that runs many groups in a fixed number of launches.
 *
 * Conventions for every entry point:
 *  - Buffers are device pointers (HBM) unless a parameter says "host".
 *    The caller owns every buffer it passes; the library never frees or
 *    retains caller memory beyond the call, and allocates nothing on the
 *    paths below except inside ne_plan_create.
 *  - A stream group is passed as a host array of M device pointers, one
 *    buffer per stream (structure of arrays). Streams within a call must not
 *    overlap unless a function says that aliasing is allowed.
 *  - `stream` is a hipStream_t (NULL is the null stream). Work is enqueued
 *    asynchronously; the library synchronises the device only in the
 *    calls documented as synchronous (ne_device_flags, ne_plan_flags). Argument
 *    errors are reported synchronously, before anything is enqueued;
 *    asynchronous HIP errors surface on a later call or on the caller's
 *    synchronisation. Calls on distinct streams are thread-safe.
 *  - Integer arithmetic on 64-bit words wraps modulo 2^64 (on 32-bit words,
 *    modulo 2^32). That is exact for this method: the admissible output
 *    range of eq. (11)/(13) guarantees every entangled output fits in the
 *    word, and wrap-around arithmetic is a ring homomorphism, so
 *    intermediate wrap-around cancels.
 *  - Lengths are element counts (int64). A length of 0 is valid and
 *    enqueues nothing; a device pointer whose buffer has length 0 is never
 *    dereferenced and may be NULL (host pointer arrays may not).
 */
#ifndef NE_H
#define NE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NE_MAX_M 32      /* largest group size accepted */
#define NE_WORD_BITS 64  /* w: width of an entangled word (the ne_*32 calls: 32) */
#define NE_MAX_M32 17    /* largest group with an admissible l at w = 32 (l = 2, k = 0) */

typedef int32_t ne_status;
#define NE_OK 0
#define NE_EINVAL (-1)    /* bad argument: M, length, NULL pointer, misuse */
#define NE_ERANGE (-2)    /* no admissible (l, k) for (M, w), or D < 1 */
#define NE_EFAILIDX (-3)  /* failed-stream index outside [-1, M) */
#define NE_EUNSUP (-4)    /* operation or shape not supported */
#define NE_EHIP (-5)      /* a HIP call failed; see ne_last_hip_error() */
#define NE_ENOMEM (-6)    /* device allocation failed (plan creation only) */
#define NE_ESCRATCH (-7)  /* needs more than the library's fixed scratch buffer
                             (ne_chain_apply_noalloc) */
#define NE_ELATE (-8)     /* more than one stream missed the deadline
                             (ne_wait_streams) */

/* The LSB operations of eq. (2) that the library runs. */
typedef enum ne_op {
    NE_OP_CONV = 0,  /* full linear convolution with a kernel g of K taps:
                        y[t] = sum_{j<K} g[j] x[t-j], 0 <= t < n+K-1 */
    NE_OP_SCALE = 1, /* y[i] = s * x[i] (scalar multiplication) */
    NE_OP_ADD = 2,   /* y[i] = x[i] + g[i] (element-wise addition) */
    NE_OP_INNER = 3, /* y[0] = sum_i x[i] g[i] (inner product) */
    NE_OP_PERM = 4,  /* y[i] = x[p[i]] for a fixed bijection p (footnote 2) */
    /* The other operators eq. (2) lists (per-step calls, series and the
       batched executor): */
    NE_OP_SUB = 5,   /* y[i] = x[i] - g[i] (element-wise subtraction) */
    NE_OP_MUL = 6,   /* y[i] = x[i] g[i] (element-by-element product) */
    NE_OP_CIRC = 7,  /* circular convolution of length n with K taps:
                        y[t] = sum_{j<K} g[j] x[(t-j) mod n], 0 <= t < n */
    NE_OP_XCORR = 8, /* full cross-correlation with K taps:
                        y[t] = sum_{j<K} g[j] x[t+j-(K-1)], 0 <= t < n+K-1 */
    NE_OP_OUTER = 9  /* outer product with a vector of K values:
                        y[i K + j] = x[i] g[j], 0 <= i < n, 0 <= j < K */
} ne_op;

typedef void *ne_stream; /* a hipStream_t */

/* Text for a status code (static storage). */
const char *ne_strerror(ne_status status);
/* The hipError_t of the most recent NE_EHIP on the calling thread, else 0. */
int32_t ne_last_hip_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t ne_version(void);

/*
 * The device flag word of the per-step calls on the calling thread's
 * current device: NE_FLAG_* bits (below) that kernels raised since the
 * last clear -- today NE_FLAG_PERM_INDEX from NE_OP_PERM. Every call
 * that uses the device shares the word, so a bit names the kind of error,
 * not the call. Synchronous: waits for all work on the device, then reads
 * (and, with clear != 0, zeroes) the word. flags: host output.
 * Errors: NE_EINVAL (NULL flags), NE_EHIP.
 */
ne_status ne_device_flags(uint32_t *flags, int32_t clear);

/*
 * Parameters (Sec. III-A eq. (8), Sec. III-B eq. (12), Table I, eq. (11),
 * eq. (13)). For M streams in w-bit words, returns the shift l, the headroom
 * k and D, the largest output magnitude the method recovers exactly:
 * outputs must satisfy |d_m[n]| <= D. l and k maximise the output
 * bit-width (M-2)l + k subject to (M-1)l + k <= w and 0 <= k <= l (larger l
 * among equals), which reproduces Table I; D follows eq. (11) for M = 3 and
 * eq. (13) for M > 3. Host-only; w in [8, 64], M in [3, NE_MAX_M].
 * Errors: NE_EINVAL (M or w outside the range, NULL outputs), NE_ERANGE
 * (eq. (13) gives D < 1). Any output pointer may be NULL except all three.
 */
ne_status ne_params(int32_t M, int32_t w, int32_t *l, int32_t *k, int64_t *dmax);

/*
 * Entangle (eq. (14)-(15)): for every position i < n and stream m < M,
 *     eps[m][i] = c[m][i] + 2^l * c[(m-1) mod M][i]      (mod 2^64).
 * c: host array of M device pointers to n int32 samples each.
 * eps: host array of M device pointers to n int64 words each (no overlap
 * with c). l in [1, 63]; normally the l of ne_params(M, 64).
 */
ne_status ne_entangle(int32_t M, int32_t l, int64_t n, const int32_t *const *c,
                      int64_t *const *eps, ne_stream stream);

/*
 * Entangle in place (the paper stores entangled data in place of the
 * inputs, Sec. II-B): x[m] holds n int64 input samples on entry and the
 * entangled words on return. Each position's M-tuple is read before any of
 * it is written.
 */
ne_status ne_entangle_inplace(int32_t M, int32_t l, int64_t n, int64_t *const *x,
                              ne_stream stream);

/*
 * Entangle an operand with itself (footnote 3), needed for NE_OP_ADD and
 * NE_OP_SUB on entangled streams: g_ent[i] = g[i] + 2^l g[i]. g: n int32; g_ent: n int64.
 */
ne_status ne_entangle_operand(int32_t l, int64_t n, const int32_t *g, int64_t *g_ent,
                              ne_stream stream);

/*
 * Run one LSB operation on each of M int64 streams independently (eq. (9)):
 *     delta[m] = eps[m] op g        for every m with bit m of stream_mask set.
 * A cleared bit models a fail-stop loss of that stream (Sec. III-B): its
 * computation is not enqueued and delta[m] is neither read nor written (and
 * may be NULL). The operation's result wraps modulo 2^64.
 *
 * op / operand / n_operand / scalar / n_out:
 *   NE_OP_CONV : operand = int32 kernel of n_operand = K >= 1 taps;
 *                n_out = n_in + K - 1 (0 when n_in = 0)
 *   NE_OP_SCALE: scalar = s (operand ignored, may be NULL); n_out = n_in
 *   NE_OP_ADD  : operand = int64 vector of n_operand = n_in words; for
 *                entangled streams it must be entangled (footnote 3,
 *                ne_entangle_operand); n_out = n_in
 *   NE_OP_INNER: operand = int32 vector of n_operand = n_in; n_out = 1
 *   NE_OP_PERM : operand = int32 indices p of n_operand = n_in, a
 *                permutation of [0, n_in); n_out = n_in. The indices live
 *                on the device and the call is asynchronous, so they are
 *                checked there: an index outside [0, n_in) reads nothing,
 *                its output is 0 and NE_FLAG_PERM_INDEX is raised in the
 *                library's device flag word (ne_device_flags). Repeated
 *                in-range indices are not detected.
 *   NE_OP_SUB  : as NE_OP_ADD (the operand entangled likewise)
 *   NE_OP_MUL  : operand = int32 vector of n_operand = n_in; n_out = n_in
 *   NE_OP_CIRC : operand = int32 kernel of K >= 1 taps (K may exceed
 *                n_in: the taps wrap); n_out = n_in
 *   NE_OP_XCORR: operand = int32 kernel of K >= 1 taps;
 *                n_out = n_in + K - 1 (0 when n_in = 0)
 *   NE_OP_OUTER: operand = int32 vector of K >= 0 values; n_out = n_in K
 * M in [1, NE_MAX_M] (the operation itself does not depend on
 * entanglement, so this also runs the checksum stream of the checksum
 * method). delta must not overlap eps or the operand.
 */
ne_status ne_lsb_apply(int32_t op, int32_t M, int64_t n_in, const int64_t *const *eps,
                       const void *operand, int64_t n_operand, int64_t scalar,
                       int64_t *const *delta, int64_t n_out, uint32_t stream_mask,
                       ne_stream stream);

/*
 * Extract and recover (eq. (16)-(19), Remark 1): from the entangled outputs
 * of the M-1 streams other than r, write all M recovered outputs
 *     dhat[m][i] = d_m[i]   for every m < M, i < n_out.
 * r is the index of the lost stream; delta[r] is never read and may be
 * NULL. r = -1 means no stream was lost; stream 0 is then left unread (every
 * choice gives the same result). l is the shift used to entangle. dhat may
 * alias delta stream by stream (dhat[m] == delta[m]): the recovery is
 * position-local and reads a position's inputs before writing its outputs.
 * Results are exact when every |d_m[i]| <= D of ne_params(M, 64).
 * Errors: NE_EFAILIDX for r outside [-1, M); NE_EINVAL for M outside
 * [3, NE_MAX_M], l outside [1, 63] or (M-1)l > 64.
 */
ne_status ne_extract_recover(int32_t M, int32_t l, int64_t n_out, const int64_t *const *delta,
                             int32_t r, int64_t *const *dhat, ne_stream stream);

/*
 * Failure-intolerant baseline: the same LSB operations on n_streams raw
 * int32 streams, int64 outputs, computed exactly (no entanglement). The
 * operand types are those of ne_lsb_apply except NE_OP_ADD and NE_OP_SUB,
 * whose operand is an int32 vector here.
 */
ne_status ne_plain_apply(int32_t op, int32_t n_streams, int64_t n_in, const int32_t *const *c,
                         const void *operand, int64_t n_operand, int64_t scalar,
                         int64_t *const *d, int64_t n_out, ne_stream stream);

/*
 * Checksum method, generation (eq. (3)-(4)): rsum[i] = sum_m c[m][i], as
 * int64. The checksum stream is then processed like the others (eq. (5)),
 * with ne_lsb_apply on one stream.
 */
ne_status ne_checksum(int32_t M, int64_t n, const int32_t *const *c, int64_t *rsum,
                      ne_stream stream);

/*
 * Checksum method, recovery of the lost output r (not printed in the paper;
 * it follows from the linearity of op on eq. (5)):
 *     d_r[i] = e[i] - sum_{m != r} d[m][i]         (mod 2^64)
 * d: host array of M device pointers (d[r] is never read and may be NULL);
 * e: the processed checksum stream; d_r: output (may alias d[r]).
 * For NE_OP_ADD the checksum stream must have been processed with the
 * operand M*g.
 */
ne_status ne_checksum_recover(int32_t M, int64_t n_out, const int64_t *const *d,
                              const int64_t *e, int32_t r, int64_t *d_r, ne_stream stream);

/*
 * Memory-bandwidth reference, none of the method's arithmetic:
 *     out[i] = in[i] (sign-extended to int64)     for i < n,
 * the HBM traffic of a fused convolution's inputs and outputs (4 bytes read
 * and 8 written per element) with the same access widths (16-byte loads,
 * non-temporal 16-byte stores). Its rate is the practical ceiling the fused
 * kernels are measured against. in and out: device memory, 16-byte aligned,
 * disjoint. Errors: NE_EINVAL (n < 0, NULL, misaligned or overlapping
 * buffers of a non-empty copy), NE_EHIP.
 */
ne_status ne_stream_widen(const int32_t *in, int64_t n, int64_t *out, ne_stream stream);

/*
 * i8 matrix-core rate reference, none of the method's arithmetic: `blocks`
 * workgroups of 4 waves each issue iters x 8 independent
 * v_mfma_i32_16x16x64_i8 on register operands, the instruction the fused
 * convolution and matrix product run. varied = 0: every product takes the
 * same operands; varied = 1: every product another pair of pseudo-random
 * operands (iters a multiple of 8), as products of data digit planes do --
 * the matrix cores' sustained rate depends on how much their operands
 * change. sink: device memory of 4 * blocks int32 (one folded word per
 * wave, so no product is dropped); ops (host, may be NULL): the integer
 * operations launched, 2 x 16 x 16 x 64 per instruction.
 * Errors: NE_EINVAL (blocks < 1, iters < 1 or not a multiple of 8 when
 * varied, NULL sink), NE_EHIP.
 */
ne_status ne_mfma_i8_peak(int32_t blocks, int64_t iters, int32_t varied, int32_t *sink,
                          double *ops, ne_stream stream);

/* ------------------------------------------------------------------------
 * Fail-stop identification by deadline (Sec. I: a failed core is
 * unresponsive or late; Sec. III-B: recovery from the M-1 streams other than
 * the unavailable one). Each entangled stream's operation runs as its own
 * task -- ne_lsb_apply with only that stream's mask bit, on its own HIP
 * stream -- followed by a completion event the caller records there.
 *
 * ne_wait_streams: waits on the host (polling, no device work) until every
 * one of the M events has completed or deadline_us microseconds have passed
 * since the call. events: host array of M hipEvent_t (as void*); a NULL
 * entry is a stream that was never launched and counts as late. *lost
 * receives the index of the one stream that had not completed by the
 * deadline, or -1 if all did; the late stream's work is neither awaited nor
 * cancelled, and recovery (ne_extract_recover with r = *lost) must not read
 * its output. The caller orders the recovery after the other M-1 events.
 * The tasks are independent failure domains only on independent hardware
 * queues: HIP streams beyond the process's hardware queues
 * (GPU_MAX_HW_QUEUES, 4 by default, read when the runtime starts) share one,
 * and a slow task then delays its queue-mates too; a process that sets it to
 * at least M before its first HIP call gives every stream its own.
 * Errors: NE_EINVAL (M outside [1, NE_MAX_M], NULL arguments, negative
 * deadline), NE_ELATE (two or more streams late: more failures than one
 * redundant stream covers; *lost = -1), NE_EHIP (an event query failed).
 *
 * ne_stream_delay: enqueues a wait of `microseconds` (at most
 * NE_MAX_DELAY_US) on `stream` -- one lane spinning on the device's
 * real-time counter -- so that work enqueued behind it completes that much
 * later: a slow core, for tests and demonstrations. Errors: NE_EINVAL
 * (negative or above the limit), NE_EHIP.
 */
#define NE_MAX_DELAY_US 1000000
ne_status ne_wait_streams(int32_t M, void *const *events, int64_t deadline_us, int32_t *lost);
ne_status ne_stream_delay(int64_t microseconds, ne_stream stream);

/* ------------------------------------------------------------------------
 * The same per-step method in 32-bit entangled words, the paper's practical
 * instantiation (Sec. III-B; Table I's w = 32 column; l = 11, k = 10 for
 * M = 3). Every entangled word, operand and recovered output is an int32,
 * so each of these calls moves half the bytes of its 64-bit counterpart.
 * Arithmetic wraps modulo 2^32, which is exact while every output satisfies
 * |d_m[i]| <= D of ne_params(M, 32) (1,046,528 for M = 3; every input
 * sample must be in that range too). Argument rules, aliasing, NULL
 * zero-length buffers and errors are those of the 64-bit calls, except
 * where stated.
 */

/* eps[m][i] = c[m][i] + 2^l c[(m-1) mod M][i] (mod 2^32), eq. (14)-(15).
 * M in [3, NE_MAX_M32]; l in [1, 31], normally the l of ne_params(M, 32). */
ne_status ne_entangle32(int32_t M, int32_t l, int64_t n, const int32_t *const *c,
                        int32_t *const *eps, ne_stream stream);

/* g_ent[i] = g[i] + 2^l g[i] (mod 2^32), footnote 3: the operand of
 * NE_OP_ADD and NE_OP_SUB on 32-bit entangled streams. */
ne_status ne_entangle_operand32(int32_t l, int64_t n, const int32_t *g, int32_t *g_ent,
                                ne_stream stream);

/* delta[m] = eps[m] op g (mod 2^32) for every m with bit m of stream_mask
 * set (eq. (9); a cleared bit is a fail-stop loss). Operation codes, shapes
 * and n_out are those of ne_lsb_apply; every operand is int32 (the entangled
 * operand of ne_entangle_operand32 for NE_OP_ADD and NE_OP_SUB); the scalar
 * of NE_OP_SCALE is taken modulo 2^32. M in [1, NE_MAX_M]. */
ne_status ne_lsb_apply32(int32_t op, int32_t M, int64_t n_in, const int32_t *const *eps,
                         const int32_t *operand, int64_t n_operand, int64_t scalar,
                         int32_t *const *delta, int64_t n_out, uint32_t stream_mask,
                         ne_stream stream);

/* Extraction and recovery (eq. (16)-(19), the register-width form of
 * Remark 1) from the int32 outputs of the M-1 streams other than r; all M
 * recovered outputs are written as int32. delta[r] is never read; r = -1
 * means no loss; dhat may alias delta stream by stream. Errors: NE_EFAILIDX
 * for r outside [-1, M); NE_EINVAL for M outside [3, NE_MAX_M32], l outside
 * [1, 31] or (M-1)l > 32. */
ne_status ne_extract_recover32(int32_t M, int32_t l, int64_t n_out, const int32_t *const *delta,
                               int32_t r, int32_t *const *dhat, ne_stream stream);

/* ------------------------------------------------------------------------
 * Series of LSB operations (Sec. II: operators applied one after another,
 * e.g. additions and scalings with fixed operands, then convolutions and
 * permutations) on the entangled streams, with one extraction at the end.
 * Every operation is linear, so after each one stream m still holds
 * d_m + 2^l d_{m-1} of the partial results; recovery needs only the last
 * stage's outputs, as for a single operation.
 */
typedef struct ne_chain_op {
    int32_t op;           /* ne_op */
    int32_t operand_bits; /* every op but NE_OP_SCALE and NE_OP_PERM: every value g
                             of the plain operand satisfies
                             -2^(b-1) <= g < 2^(b-1), b in [1, 32] (the
                             range check's promise; not verified on the
                             device); ignored for NE_OP_SCALE and NE_OP_PERM */
    const void *operand;  /* device operand, typed as for ne_lsb_apply (for
                             NE_OP_ADD and NE_OP_SUB on entangled streams:
                             the entangled int64 vector,
                             ne_entangle_operand); may be NULL
                             for ne_chain_check, which reads no operand */
    int64_t n_operand;    /* taps (conv, circ, xcorr), values (outer); the
                             current length (add, sub, mul, inner, perm);
                             ignored for scale */
    int64_t scalar;       /* NE_OP_SCALE: the factor */
} ne_chain_op;

/*
 * Shapes and worst-case range of a series on M streams of n_in samples
 * whose values lie in [-2^(in_bits-1), 2^(in_bits-1)). Stage by stage, the
 * bound B on |d| becomes K 2^(b-1) B (conv, circ, xcorr), |s| B (scale),
 * B + 2^(b-1) (add, sub), n 2^(b-1) B (inner), 2^(b-1) B (mul, outer) or
 * B (perm); every stage must satisfy
 * B <= D of ne_params(M, 64), so that no entangled intermediate leaves the
 * 64-bit range (wrapping would be harmless for these linear operations,
 * but the check keeps every intermediate an exact integer). Host-only.
 * Outputs (either may be NULL): n_out, the last stage's length; bound, the
 * last stage's B.
 * Errors: NE_EINVAL (M outside [3, NE_MAX_M], in_bits outside [1, 32],
 * n_ops outside [1, 64], n_in < 0, NULL ops, operand_bits outside [1, 32]
 * where used, an operand length that does not match), NE_EUNSUP (unknown
 * op), NE_ERANGE (a stage's bound above D).
 */
ne_status ne_chain_check(int32_t M, int32_t in_bits, int64_t n_in, const ne_chain_op *ops,
                         int32_t n_ops, int64_t *n_out, int64_t *bound);

/*
 * Bytes of device workspace ne_chain_apply needs for a series: two buffers
 * of M int64 streams of the longest intermediate length (0 for one
 * operation). Host-only; errors as ne_chain_check, without the range.
 */
ne_status ne_chain_workspace_size(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                  int32_t n_ops, size_t *bytes);

/*
 * Run the series on each of M int64 streams independently:
 *     delta[m] = (...((eps[m] op_0 g_0) op_1 g_1) ...) op_{n_ops-1} g_{n_ops-1}
 * for every m with bit m of stream_mask set (a cleared bit: a fail-stop
 * loss of that stream's core for the whole series; delta[m] is neither
 * read nor written and may be NULL). Intermediates go to the caller's
 * workspace (ne_chain_workspace_size bytes, 256-byte aligned, device
 * memory; may be NULL when that size is 0); results wrap modulo 2^64.
 * n_out must be the series' output length. Launches on `stream` only, no
 * allocation. delta must not overlap eps, the operands or the workspace.
 * Errors: as ne_chain_workspace_size, and NE_EINVAL for a missing or small
 * workspace, a wrong n_out or NULL pointers of computed streams.
 */
ne_status ne_chain_apply(int32_t M, int64_t n_in, const int64_t *const *eps,
                         const ne_chain_op *ops, int32_t n_ops, int64_t *const *delta,
                         int64_t n_out, uint32_t stream_mask, void *workspace,
                         size_t workspace_bytes, ne_stream stream);

/*
 * The whole method on a series (Sec. II: entangle once, the operators one
 * after another, extract once): entangle the M int32 streams c with l of
 * ne_params(M, 64), run the series on every stream but `lost` (-1: none
 * lost, every stream runs), extract and recover all M outputs into dhat
 * (int64, n_out each):
 *     dhat[m] = (...((c[m] op_0 g_0) op_1 g_1) ...) op_{n_ops-1} g_{n_ops-1}.
 * Stages as in ne_chain_apply; in addition the entanglement is done on load
 * by the first stage when it is a run of element-wise operations (or a
 * permutation), and the recovery by the last stage when it is one (the
 * whole series in one pass when it is a single such run); otherwise they
 * are passes of their own. Operands as for ne_chain_apply (add and sub:
 * entangled int64 words, ne_entangle_operand). The range is the caller's
 * promise (ne_chain_check). Workspace: ne_chain_run_workspace_size bytes,
 * 256-byte aligned device memory (NULL when that size is 0). dhat must not
 * overlap c, the operands or the workspace. Launches on `stream` only, no
 * allocation; a permutation index outside [0, n) raises NE_FLAG_PERM_INDEX
 * (ne_device_flags) and reads nothing.
 * Errors: NE_EINVAL (M outside [3, NE_MAX_M], a wrong n_out, NULL pointers,
 * a missing, small or misaligned workspace, and as ne_chain_workspace_size),
 * NE_EFAILIDX (lost outside [-1, M)), NE_EUNSUP (unknown op), NE_ERANGE (no
 * admissible l for M at w = 64).
 */
ne_status ne_chain_run_workspace_size(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                      int32_t n_ops, size_t *bytes);
ne_status ne_chain_run(int32_t M, int64_t n_in, const int32_t *const *c, const ne_chain_op *ops,
                       int32_t n_ops, int32_t lost, int64_t *const *dhat, int64_t n_out,
                       void *workspace, size_t workspace_bytes, ne_stream stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * series as ne_chain_apply, with the intermediates in a fixed buffer that
 * the library holds in device memory instead of caller workspace. The
 * buffer is NE_CHAIN_SCRATCH_BYTES on every device the library runs on (a
 * static device array, held until the process ends); the call allocates
 * nothing and launches on `stream` only. Every call on one device shares
 * that device's buffer: calls that overlap in time on one device (other
 * streams or threads) race on it and must be serialised by the caller; each
 * stage writes every intermediate it later reads, so nothing in the buffer
 * needs clearing. Arguments as ne_chain_apply without the workspace.
 * Errors: as ne_chain_apply (checked before the device is touched), and
 * NE_ESCRATCH when ne_chain_workspace_size for these arguments exceeds
 * NE_CHAIN_SCRATCH_BYTES (e.g. a series of two or more stages on three
 * streams longer than about 1.4 million samples).
 */
#define NE_CHAIN_SCRATCH_BYTES ((size_t)64 << 20)
ne_status ne_chain_apply_noalloc(int32_t M, int64_t n_in, const int64_t *const *eps,
                                 const ne_chain_op *ops, int32_t n_ops, int64_t *const *delta,
                                 int64_t n_out, uint32_t stream_mask, ne_stream stream);

/*
 * The same series in 32-bit entangled words (the paper's practical w = 32):
 * ne_chain_check32 bounds every stage by D of ne_params(M, 32) (M in
 * [3, NE_MAX_M32]); ne_chain_workspace_size32 counts int32 intermediates;
 * ne_chain_apply32 runs the series on int32 streams modulo 2^32 with the
 * operations of ne_lsb_apply32 (every operand int32; an added or
 * subtracted vector entangled by ne_entangle_operand32). ne_chain_run32
 * (+ ne_chain_run_workspace_size32) is ne_chain_run in these words: int32
 * samples in, int32 recovered outputs out (|d| <= D of ne_params(M, 32)),
 * l of ne_params(M, 32), the same passes. Arguments and errors otherwise
 * as the 64-bit calls.
 */
ne_status ne_chain_check32(int32_t M, int32_t in_bits, int64_t n_in, const ne_chain_op *ops,
                           int32_t n_ops, int64_t *n_out, int64_t *bound);
ne_status ne_chain_workspace_size32(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                    int32_t n_ops, size_t *bytes);
ne_status ne_chain_apply32(int32_t M, int64_t n_in, const int32_t *const *eps,
                           const ne_chain_op *ops, int32_t n_ops, int32_t *const *delta,
                           int64_t n_out, uint32_t stream_mask, void *workspace,
                           size_t workspace_bytes, ne_stream stream);
ne_status ne_chain_run_workspace_size32(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                        int32_t n_ops, size_t *bytes);
ne_status ne_chain_run32(int32_t M, int64_t n_in, const int32_t *const *c, const ne_chain_op *ops,
                         int32_t n_ops, int32_t lost, int32_t *const *dhat, int64_t n_out,
                         void *workspace, size_t workspace_bytes, ne_stream stream);

/* ------------------------------------------------------------------------
 * Entangled integer matrix product: the multiplication operator of eq. (2)
 * applied to M blocks of the streams and one shared kernel matrix (the GEMM
 * case of Sec. IV, eq. (20)): D_m = C_m G for every block m, computed by the
 * method of `mode` in one fused pass -- blocks entangled on load
 * (eq. (14)-(15)), each entangled block multiplied by G on the i8 matrix
 * cores, every output recovered from the M-1 blocks other than `lost`
 * (eq. (16)-(19)) -- or plain, plain on the same datapath, or with a
 * checksum block (eq. (3)-(5)).
 *
 * c: host array of M device pointers to N x P int32 matrices (row-major);
 * g: device P x Q int32 matrix (row-major); out: host array of M device
 * pointers to N x Q int64 matrices (row-major, disjoint from the inputs).
 * Every value of c and g must lie in [-2^(in_bits-1), 2^(in_bits-1)),
 * in_bits in [1, 16]; values outside are flagged (NE_FLAG_INPUT_RANGE).
 * lost: -1, or the block whose product is not computed (its output is
 * recovered; plain modes leave it unwritten). flags: device word OR-ed with
 * NE_FLAG_* bits (NULL: not reported). No allocation; launches on `stream`
 * only.
 * workspace: NULL runs one fused launch (digits split in LDS inside the
 * product kernel, recovery in registers; with no loss the redundant block
 * is checked, NE_FLAG_MISMATCH). Otherwise device memory of
 * ne_gemm_workspace_size bytes, 256-byte aligned, owned by the caller: the
 * digit planes of every block's (entangled) values and of G are written
 * there once; every computed block's product is then an independent slice
 * of one launch reading its matrix-core fragments straight from the planes
 * and writing its entangled outputs into that block's output buffer (the
 * checksum block's into the workspace); recovery follows in place (no
 * redundancy check). Faster for large products.
 * Errors: NE_EINVAL (mode, M, negative sizes, NULL pointers of non-empty
 * matrices, a short or misaligned workspace), NE_EFAILIDX (lost), NE_ERANGE (P 2^(2 in_bits - 2) above D of
 * ne_params(M, 64) for the method, above 2^63 - 1 otherwise), NE_EUNSUP
 * (in_bits above 16, N above 32 * 65535, Q above 2^26, P above 2^24, or an
 * inner dimension too long for exact 32-bit digit sums).
 */
ne_status ne_gemm(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q,
                  const int32_t *const *c, const int32_t *g, int64_t *const *out, int32_t lost,
                  int32_t in_bits, void *workspace, size_t workspace_bytes, uint32_t *flags,
                  ne_stream stream);

/*
 * Workspace bytes of ne_gemm's two-phase form for these arguments (0 when
 * there is no output). Host-only; errors as ne_gemm's argument checks.
 */
ne_status ne_gemm_workspace_size(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q,
                                 int32_t in_bits, size_t *bytes);

/* ------------------------------------------------------------------------
 * Batched executor: many groups (uneven M, length, operation and operand
 * size) in a fixed set of fused launches, optionally as one hipGraph.
 *
 * In NE_MODE_ENTANGLED each group goes through the whole method in one pass
 * over HBM: its int32 inputs are read once, entangled on load (eq. (14)-
 * (15)), the operation runs on every entangled stream (eq. (9); convolution
 * on the i8 matrix cores with exact digit splitting, the others on the
 * vector ALUs), and the outputs are recovered from the M-1 streams other
 * than the lost one (eq. (16)-(19)) before anything is written; only the
 * recovered int64 outputs reach memory. The lost stream's operation is not
 * run. When no stream is lost, the redundant stream is checked against the
 * recovered outputs and a disagreement sets NE_FLAG_MISMATCH.
 *
 * The other modes run the baselines on the same machinery: NE_MODE_PLAIN is
 * the failure-intolerant operation with the fewest digits the declared
 * input range needs; NE_MODE_PLAIN_SAME the same operation on the datapath
 * (digit counts) the entangled words need; NE_MODE_CHECKSUM the checksum
 * method of eq. (3)-(5) (M data streams plus their sum, with recovery of a
 * lost stream as d_r = e - sum of the others), with the fewest digits the
 * sum stream needs; NE_MODE_CHECKSUM_SAME the checksum method on the
 * entangled words' datapath (the paper's comparison ran every variant
 * through one routine, Sec. V). Element-wise operations have one datapath,
 * so the two checksum modes and the two plain modes coincide for them.
 *
 * Digits of a convolution: the inputs and taps are cut into balanced
 * base-256 digits for the i8 matrix cores. Where it takes fewer digit planes,
 * every data word x is first split at bit l into a balanced low field lo and
 * a high field hi = (x - lo) / 2^l, each with its own digits (an entangled
 * word of 12-bit samples at M = 3: 2 + 2 digits instead of 5); the split is
 * computed from x alone, so each stream's product still depends only on its
 * own entangled input.
 * ------------------------------------------------------------------------ */

#define NE_FUSED_MAX_M 8

typedef enum ne_mode {
    NE_MODE_ENTANGLED = 0,
    NE_MODE_PLAIN = 1,
    NE_MODE_PLAIN_SAME = 2,
    NE_MODE_CHECKSUM = 3,
    NE_MODE_CHECKSUM_SAME = 4
} ne_mode;

/* Device-side error bits (ne_plan_flags). */
#define NE_FLAG_INPUT_RANGE 1u /* an input or operand value outside in_bits */
#define NE_FLAG_LIMBS 2u       /* reserved, never raised: digit counts follow
                                  in_bits, which every input is checked against */
#define NE_FLAG_MISMATCH 4u    /* redundant stream disagrees with the outputs */
#define NE_FLAG_PERM_INDEX 8u  /* a permutation index outside [0, n): that
                                  output is undefined (ne_plan_flags) or 0
                                  (the per-step calls, ne_device_flags) */
#define NE_FLAG_STALL 16u      /* single launch: a permutation's gathers waited
                                  past their bound for its layout pass; its
                                  outputs are undefined */

/* One group: M streams of n int32 samples sharing one operand. */
typedef struct ne_group {
    int32_t op;          /* ne_op: any of the ten */
    int32_t M;           /* streams: 3..8 (entangled), 2..8 (checksum), 1..8 */
    int64_t n;           /* samples per stream (>= 0) */
    int64_t n_operand;   /* K taps (conv, circ, xcorr), K values (outer: n K
                            outputs), n (add, sub, mul, inner, perm), 0 (scale) */
    int64_t scalar;      /* scale factor (NE_OP_SCALE) */
    int32_t lost;        /* -1, or the stream whose operation is dropped */
    int32_t in_bits;     /* 1..31 (conv, circ, xcorr) or 1..32: every sample and operand
                            value v satisfies -2^(in_bits-1) <= v < 2^(in_bits-1);
                            violations are flagged (NE_FLAG_INPUT_RANGE) */
    int32_t steps;       /* tile steps per block for this group (conv: 1024
                            outputs each; element-wise: see ne_tuning); 0: the
                            plan's ne_tuning value */
    int32_t ring_waves;  /* conv: waves that share one staging ring: 4 (one
                            ring per block of 4 waves, two block barriers per
                            step) or 1 (a ring per wave, no barrier in the
                            step loop); 0: the plan's choice */
    int32_t tap_copies;  /* conv: copies of each tap-digit plane in LDS: 4
                            (one per byte alignment, every operand fragment
                            read aligned) or 1 (a quarter of the LDS, each
                            fragment realigned in registers; block rings
                            only, for long kernels); 0: the plan's choice (1
                            only where it fits more blocks per CU than 4, or
                            4 does not fit at all) */
    int32_t word_bits;   /* w, the width of the entangled words: 0 or 64
                            (outputs int64, D of ne_params(M, 64)), or 32
                            (the paper's practical width: l and D of
                            ne_params(M, 32), outputs stored as int32; plain
                            and checksum groups: results within 2^31 - 1) */
    const int32_t *c[NE_FUSED_MAX_M]; /* device inputs; 16-byte aligned */
    const int32_t *operand;           /* device int32 taps / vector /
                                         permutation indices, 16-byte aligned;
                                         NULL for scale.
                                         For add and sub, the plain vector g
                                         (the entangled mode entangles it
                                         itself, footnote 3). */
    void *out[NE_FUSED_MAX_M];        /* device outputs, n_out int64 each
                                         (int32 with word_bits = 32),
                                         16-byte aligned, disjoint */
} ne_group;

typedef struct ne_tuning {
    int32_t conv_steps;   /* 1024-output steps per convolution block; 0: 4 */
    int32_t stream_steps; /* steps of 256 lanes x 4 (M <= 4) or x 2 positions
                             per element-wise block; 0: 4 */
    int32_t single_launch; /* 0: one launch per kernel variant (a captured run
                             spreads them over parallel graph branches);
                             1: the whole run is one persistent launch whose
                             blocks take the plan's work items from a device
                             queue: permutation layout passes first, then
                             the convolutions (longest first) interleaved
                             with the permutation gathers, then the other
                             element-wise items; each item at least 4 tile
                             steps long.
                             Its menu: conv, circ and xcorr groups of 3..8
                             data streams with in_bits 9..12 (the digit counts
                             those take), scale, add, inner and perm groups of
                             3..8 data streams; any other group makes plan
                             creation fail with NE_EUNSUP. The queue and the
                             per-group counters return to zero within each
                             run: a run that did not complete leaves the plan
                             unusable (destroy it and build it again). */
} ne_tuning;

typedef struct ne_plan_stats {
    int64_t groups, items, launches;
    int64_t in_bytes;     /* int32 input and operand bytes one run must read */
    int64_t out_bytes;    /* output bytes one run must write */
    int64_t out_samples;  /* recovered output samples of one run */
    int64_t macs;         /* useful multiply-adds of one run (conv and inner) */
    int64_t mfma_macs;    /* i8 multiply-adds issued on the matrix cores */
    int64_t lds_bytes;    /* largest dynamic LDS of a launch */
    int64_t limb_macs;    /* useful convolution multiply-adds x the digit pairs each
                             takes on the matrix cores (mfma_macs without the
                             Toeplitz padding and the data-dependent sparse digit) */
} ne_plan_stats;

typedef struct ne_plan ne_plan;

/*
 * Validate the groups (host array of n_groups), choose digit counts from
 * in_bits, check that every group's worst-case output is admissible
 * (|d| <= D of eq. (11)/(13) for the group's word width in
 * NE_MODE_ENTANGLED, |d| < 2^(w-1) otherwise; NE_ERANGE if not), build the work items and upload them. Allocates device
 * memory for the plan only (freed by ne_plan_destroy): its tables, plus, per
 * permutation group, n rows of 16 (at most 4 slots) or 32 bytes into which
 * every run first interleaves the group's streams (so that each gather at
 * pi[i] reads one row). The caller keeps
 * owning every buffer the groups point to; they must stay valid while the
 * plan is used. tuning may be NULL.
 */
ne_status ne_plan_create(const ne_group *groups, int32_t n_groups, int32_t mode,
                         const ne_tuning *tuning, ne_plan **plan);
/*
 * Device bytes a plan over these groups needs when the caller provides the
 * memory (ne_plan_create_in). Host-only; validates like ne_plan_create.
 */
ne_status ne_plan_workspace_size(const ne_group *groups, int32_t n_groups, int32_t mode,
                                 const ne_tuning *tuning, size_t *bytes);
/*
 * ne_plan_create without any device allocation or synchronisation: the plan
 * tables live in the caller's `workspace` (device memory, 256-byte aligned,
 * at least ne_plan_workspace_size bytes) and are uploaded asynchronously on
 * `stream`; the plan must be run on that stream (or after it). For callers
 * that run many short plans concurrently (serving): ne_plan_destroy then only
 * frees host memory, and must be called only after `stream` has completed the
 * upload (for example after the plan's last run has completed).
 */
ne_status ne_plan_create_in(const ne_group *groups, int32_t n_groups, int32_t mode,
                            const ne_tuning *tuning, void *workspace, size_t workspace_bytes,
                            ne_stream stream, ne_plan **plan);
/* Enqueue one run of the whole batch on `stream`. Allocates nothing. Runs of
 * one plan must not overlap in time (issue them on one stream, or order them
 * with events): they share the plan's accumulators, permutation rows and, with
 * single_launch, its work queue and counters. Different plans are independent. */
ne_status ne_plan_run(ne_plan *plan, ne_stream stream);
/* Record one run into a hipGraph (by stream capture on `stream`); later
 * ne_plan_launch calls replay it as one graph launch. */
ne_status ne_plan_capture(ne_plan *plan, ne_stream stream);
/* Launch the captured graph (or enqueue a run if none was captured). */
ne_status ne_plan_launch(ne_plan *plan, ne_stream stream);
/* Synchronously read (and optionally clear) the device error bits. */
ne_status ne_plan_flags(ne_plan *plan, uint32_t *flags, int32_t clear);
ne_status ne_plan_stats_get(const ne_plan *plan, ne_plan_stats *stats);
ne_status ne_plan_destroy(ne_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* NE_H */
