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
 *      held in 64-bit words (w = 64);
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
 *    asynchronously; the library never synchronises the device. Argument
 *    errors are reported synchronously, before anything is enqueued;
 *    asynchronous HIP errors surface on a later call or on the caller's
 *    synchronisation. Calls on distinct streams are thread-safe.
 *  - Integer arithmetic on 64-bit words wraps modulo 2^64. That is exact for
 *    this method: the admissible output range of eq. (11)/(13) guarantees
 *    every entangled output fits in 64 bits, and wrap-around arithmetic is a
 *    ring homomorphism, so intermediate wrap-around cancels.
 *  - Lengths are element counts (int64). A length of 0 is valid and
 *    enqueues nothing.
 */
#ifndef NE_H
#define NE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NE_MAX_M 32      /* largest group size accepted */
#define NE_WORD_BITS 64  /* w: width of an entangled word */

typedef int32_t ne_status;
#define NE_OK 0
#define NE_EINVAL (-1)    /* bad argument: M, length, NULL pointer, misuse */
#define NE_ERANGE (-2)    /* no admissible (l, k) for (M, w), or D < 1 */
#define NE_EFAILIDX (-3)  /* failed-stream index outside [-1, M) */
#define NE_EUNSUP (-4)    /* operation or shape not supported */
#define NE_EHIP (-5)      /* a HIP call failed; see ne_last_hip_error() */
#define NE_ENOMEM (-6)    /* device allocation failed (plan creation only) */

/* The LSB operations of eq. (2) that the library runs. */
typedef enum ne_op {
    NE_OP_CONV = 0,  /* full linear convolution with a kernel g of K taps:
                        y[t] = sum_{j<K} g[j] x[t-j], 0 <= t < n+K-1 */
    NE_OP_SCALE = 1, /* y[i] = s * x[i] (scalar multiplication) */
    NE_OP_ADD = 2,   /* y[i] = x[i] + g[i] (element-wise addition) */
    NE_OP_INNER = 3, /* y[0] = sum_i x[i] g[i] (inner product) */
    NE_OP_PERM = 4   /* y[i] = x[p[i]] for a fixed bijection p (footnote 2) */
} ne_op;

typedef void *ne_stream; /* a hipStream_t */

/* Text for a status code (static storage). */
const char *ne_strerror(ne_status status);
/* The hipError_t of the most recent NE_EHIP on the calling thread, else 0. */
int32_t ne_last_hip_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t ne_version(void);

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
 * Entangle an operand with itself (footnote 3), needed for NE_OP_ADD on
 * entangled streams: g_ent[i] = g[i] + 2^l g[i]. g: n int32; g_ent: n int64.
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
 *                permutation of [0, n_in) (not checked; an index outside
 *                the range is clamped into it); n_out = n_in
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
 * operand types are those of ne_lsb_apply except NE_OP_ADD, whose operand
 * is an int32 vector here.
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

#ifdef __cplusplus
}
#endif
#endif /* NE_H */
