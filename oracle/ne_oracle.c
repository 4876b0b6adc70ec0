/*
 * Plain, slow CPU oracle for numerical entanglement of integer streams
 * (Anam & Andreopoulos, "Failure Mitigation in Linear, Sesquilinear and
 * Bijective Operations On Integer Data Streams Via Numerical Entanglement",
 * IOLTS 2015).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library shares no
 * code, header or table with it, and this file includes nothing from it.
 *
 * Every value is carried in a 128-bit signed integer and every add, multiply
 * and shift that could leave that range is checked, so a result is either
 * the exact integer the paper defines or an error code. A "w-bit register" is
 * modelled explicitly: entangled words must fit in w bits (eq. (8)/(12) are
 * there to guarantee that), and the extraction temporary lives in a 2w-bit
 * register as Sec. III-A and eq. (16) state.
 *
 * Data layout: a group of M streams of n samples is one row-major array
 * x[m*n + i]. Outputs are int64 (w <= 64).
 *
 * Parity pins: every function here is checked in the test suite against
 * something other than itself (Table I, the textbook definitions of the LSB
 * operations through numpy, exhaustive enumeration of the admissible output
 * range at tiny w, the closed form of the entangled outputs, and the
 * all-subsets invariant). None of the result is "parity unpinned".
 */
#include <stdint.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1,   /* bad argument */
    ORC_EOVERFLOW = 2,/* a value left the w-bit (or 2w-bit) register */
    ORC_EINEXACT = 3  /* a shift that the method says is exact dropped bits */
};

enum {
    ORC_CONV = 0, ORC_SCALE = 1, ORC_ADD = 2, ORC_INNER = 3, ORC_PERM = 4,
    ORC_SUB = 5, ORC_MUL = 6, ORC_CIRC = 7, ORC_XCORR = 8, ORC_OUTER = 9
};

/* ---------------------------------------------------------------- helpers */

/* Does x fit in a signed two's-complement register of `bits` bits? */
static int fits(i128 x, int bits)
{
    if (bits >= 128) return 1;
    i128 hi = ((i128)1 << (bits - 1)) - 1;
    i128 lo = -((i128)1 << (bits - 1));
    return x >= lo && x <= hi;
}

/* Reduce x modulo 2^bits into the signed range of a `bits`-bit register
 * (two's-complement truncation at the most significant bit, footnote 1). */
static i128 wrap(i128 x, int bits)
{
    if (bits >= 128) return x;
    u128 mask = (((u128)1) << bits) - 1;
    u128 u = ((u128)x) & mask;
    if (u >> (bits - 1)) u |= ~mask; /* sign bit set: extend it */
    return (i128)u;
}

/* The shift operator S_l of eq. (7) acting on a `bits`-bit register:
 * l >= 0 shifts left, truncating at the most significant bit of the
 * register; l < 0 shifts right arithmetically by -l, truncating the least
 * significant bits (footnote 1). gcc documents >> on negative signed
 * integers as arithmetic. */
static i128 S(i128 x, int l, int bits)
{
    if (l >= 0) {
        if (l >= 128) return 0;
        return wrap((i128)(((u128)x) << l), bits);
    }
    int r = -l;
    if (r >= 127) return x < 0 ? -1 : 0;
    return x >> r;
}

static int add_ok(i128 a, i128 b, i128 *out) { return !__builtin_add_overflow(a, b, out); }
static int mul_ok(i128 a, i128 b, i128 *out) { return !__builtin_mul_overflow(a, b, out); }

/* ------------------------------------------------------------ parameters */

/* Choice of l and k (eq. (8) for M = 3, eq. (12) in general, Table I).
 * Among all integers l >= 1, 0 <= k <= l with (M-1)l + k <= w, take the pair
 * with the largest output bit-width (M-2)l + k -- the quantity Table I
 * tabulates -- and among equals the larger l. This reproduces all seven rows
 * of Table I and, for M = 3, coincides with "l + k maximal, k <= l".
 * D is the largest admissible output magnitude: eq. (11) for M = 3,
 * eq. (13) for M >= 4. Returns ORC_EINVAL when no pair exists. */
int orc_params(int M, int w, int *l_out, int *k_out, int64_t *dmax_out)
{
    if (M < 3 || w < 4 || w > 64) return ORC_EINVAL;
    int best_l = -1, best_k = -1, best_obj = -1;
    for (int l = 1; l <= w; ++l) {
        for (int k = 0; k <= l; ++k) {
            if ((M - 1) * l + k > w) continue;
            int obj = (M - 2) * l + k;
            if (obj > best_obj || (obj == best_obj && l > best_l)) {
                best_obj = obj; best_l = l; best_k = k;
            }
        }
    }
    if (best_l < 0) return ORC_EINVAL;
    int l = best_l, k = best_k;
    i128 D;
    if (M == 3) {
        /* eq. (11): |d| <= 2^(l+k-1) - 2^l */
        D = ((i128)1 << (l + k - 1)) - ((i128)1 << l);
    } else {
        /* eq. (13): |d| <= 2^((M-3)l+k) * (2^(l-1) - 1) */
        D = ((i128)1 << ((M - 3) * l + k)) * (((i128)1 << (l - 1)) - 1);
    }
    if (l_out) *l_out = l;
    if (k_out) *k_out = k;
    if (dmax_out) *dmax_out = (int64_t)D;
    /* D may be 0: eq. (13) gives an empty range when l = 1 (e.g. the M = 32
     * row of Table I). l and k are still reported; callers reject D < 1. */
    return ORC_OK;
}

/* ----------------------------------------------------------- entanglement */

/* eq. (14)-(15): per position n, the entangled vector is E applied to the
 * M-vector of inputs, E circulant with first row [1 0 ... 0 S_l]; row m has
 * the 1 in column m and S_l in column (m-1) mod M, i.e.
 *     eps_m = c_m + S_l{c_{(m-1) mod M}}      (eq. (6) for M = 3).
 * The result must fit in w bits; otherwise ORC_EOVERFLOW. */
int orc_entangle(int M, int l, int w, int64_t n, const int64_t *c, int64_t *eps)
{
    if (M < 3 || l < 1 || w < 2 || w > 64 || n < 0) return ORC_EINVAL;
    for (int m = 0; m < M; ++m) {
        int prev = (m - 1 + M) % M;
        for (int64_t i = 0; i < n; ++i) {
            i128 shifted;
            if (!mul_ok((i128)c[prev * n + i], (i128)1 << l, &shifted)) return ORC_EOVERFLOW;
            i128 e = (i128)c[m * n + i] + shifted;
            if (!fits(e, w)) return ORC_EOVERFLOW;
            eps[m * n + i] = (int64_t)e;
        }
    }
    return ORC_OK;
}

/* Footnote 3: for op in {+, -} the operand is entangled with itself,
 * g_n <- S_l{g_n} + g_n, so that the addition stays a homomorphism. */
int orc_entangle_operand(int l, int w, int64_t n, const int64_t *g, int64_t *gent)
{
    if (l < 1 || w < 2 || w > 64 || n < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        i128 shifted;
        if (!mul_ok((i128)g[i], (i128)1 << l, &shifted)) return ORC_EOVERFLOW;
        i128 e = shifted + (i128)g[i];
        if (!fits(e, w)) return ORC_EOVERFLOW;
        gent[i] = (int64_t)e;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------- LSB ops */

/* One output of the full linear convolution of x (length n) with g
 * (length K): y[t] = sum_{j=0}^{K-1} g[j] * x[t-j], x zero outside [0, n).
 * This is convolution (kernel reversed against the data), not correlation. */
static int conv_one(const int64_t *x, int64_t n, const int64_t *g, int64_t K, int64_t t, i128 *out)
{
    i128 acc = 0;
    for (int64_t j = 0; j < K; ++j) {
        int64_t src = t - j;
        if (src < 0 || src >= n) continue;
        i128 p;
        if (!mul_ok((i128)g[j], (i128)x[src], &p)) return 0;
        if (!add_ok(acc, p, &acc)) return 0;
    }
    *out = acc;
    return 1;
}

/* d = x op g for one stream, eq. (2) and eq. (9), computed exactly.
 *   ORC_CONV : full linear convolution, n_out = n_in + n_operand - 1
 *              (n_out = 0 when either length is 0)
 *   ORC_SCALE: d[i] = scalar * x[i], n_out = n_in
 *   ORC_ADD  : d[i] = x[i] + operand[i], n_out = n_in = n_operand
 *              (on entangled data the operand must be entangled first,
 *               footnote 3)
 *   ORC_INNER: d[0] = sum_i x[i] * operand[i], n_out = 1, n_operand = n_in
 *   ORC_PERM : d[i] = x[operand[i]], a fixed bijection of [0, n_in)
 *              (footnote 2), n_out = n_in = n_operand
 * and the other operators eq. (2) lists:
 *   ORC_SUB  : d[i] = x[i] - operand[i] (entangled operand on entangled
 *              data, as for addition)
 *   ORC_MUL  : d[i] = x[i] * operand[i] (element-by-element product)
 *   ORC_CIRC : circular convolution of length n_in,
 *              d[t] = sum_j operand[j] x[(t - j) mod n_in], n_out = n_in
 *   ORC_XCORR: full cross-correlation,
 *              d[t] = sum_j operand[j] x[t + j - (n_operand - 1)],
 *              n_out = n_in + n_operand - 1 (0 when either length is 0)
 *   ORC_OUTER: outer product, d[i n_operand + j] = x[i] operand[j],
 *              n_out = n_in n_operand
 * Every output must fit in w bits, else ORC_EOVERFLOW. */
int orc_op(int op, int w, int64_t n_in, const int64_t *x, const int64_t *operand,
           int64_t n_operand, int64_t scalar, int64_t *out, int64_t n_out)
{
    if (w < 2 || w > 64 || n_in < 0 || n_operand < 0 || n_out < 0) return ORC_EINVAL;
    switch (op) {
    case ORC_CONV: {
        int64_t want = (n_in == 0 || n_operand == 0) ? 0 : n_in + n_operand - 1;
        if (n_out != want) return ORC_EINVAL;
        for (int64_t t = 0; t < n_out; ++t) {
            i128 v;
            if (!conv_one(x, n_in, operand, n_operand, t, &v)) return ORC_EOVERFLOW;
            if (!fits(v, w)) return ORC_EOVERFLOW;
            out[t] = (int64_t)v;
        }
        return ORC_OK;
    }
    case ORC_SCALE: {
        if (n_out != n_in) return ORC_EINVAL;
        for (int64_t i = 0; i < n_in; ++i) {
            i128 v;
            if (!mul_ok((i128)scalar, (i128)x[i], &v) || !fits(v, w)) return ORC_EOVERFLOW;
            out[i] = (int64_t)v;
        }
        return ORC_OK;
    }
    case ORC_ADD: {
        if (n_out != n_in || n_operand != n_in) return ORC_EINVAL;
        for (int64_t i = 0; i < n_in; ++i) {
            i128 v = (i128)x[i] + (i128)operand[i];
            if (!fits(v, w)) return ORC_EOVERFLOW;
            out[i] = (int64_t)v;
        }
        return ORC_OK;
    }
    case ORC_INNER: {
        if (n_out != 1 || n_operand != n_in) return ORC_EINVAL;
        i128 acc = 0;
        for (int64_t i = 0; i < n_in; ++i) {
            i128 p;
            if (!mul_ok((i128)x[i], (i128)operand[i], &p) || !add_ok(acc, p, &acc))
                return ORC_EOVERFLOW;
        }
        if (!fits(acc, w)) return ORC_EOVERFLOW;
        out[0] = (int64_t)acc;
        return ORC_OK;
    }
    case ORC_PERM: {
        if (n_out != n_in || n_operand != n_in) return ORC_EINVAL;
        for (int64_t i = 0; i < n_in; ++i) {
            int64_t s = operand[i];
            if (s < 0 || s >= n_in) return ORC_EINVAL;
            out[i] = x[s];
        }
        return ORC_OK;
    }
    case ORC_SUB:
    case ORC_MUL: {
        if (n_out != n_in || n_operand != n_in) return ORC_EINVAL;
        for (int64_t i = 0; i < n_in; ++i) {
            i128 v;
            if (op == ORC_SUB)
                v = (i128)x[i] - (i128)operand[i];
            else if (!mul_ok((i128)x[i], (i128)operand[i], &v))
                return ORC_EOVERFLOW;
            if (!fits(v, w)) return ORC_EOVERFLOW;
            out[i] = (int64_t)v;
        }
        return ORC_OK;
    }
    case ORC_CIRC: {
        if (n_out != n_in || (n_in > 0 && n_operand < 1)) return ORC_EINVAL;
        for (int64_t t = 0; t < n_out; ++t) {
            i128 acc = 0, p;
            for (int64_t j = 0; j < n_operand; ++j) {
                int64_t src = (t - j) % n_in;
                if (src < 0) src += n_in;
                if (!mul_ok((i128)operand[j], (i128)x[src], &p) || !add_ok(acc, p, &acc))
                    return ORC_EOVERFLOW;
            }
            if (!fits(acc, w)) return ORC_EOVERFLOW;
            out[t] = (int64_t)acc;
        }
        return ORC_OK;
    }
    case ORC_XCORR: {
        int64_t want = (n_in == 0 || n_operand == 0) ? 0 : n_in + n_operand - 1;
        if (n_out != want) return ORC_EINVAL;
        for (int64_t t = 0; t < n_out; ++t) {
            i128 acc = 0, p;
            for (int64_t j = 0; j < n_operand; ++j) {
                int64_t src = t + j - (n_operand - 1);
                if (src < 0 || src >= n_in) continue;
                if (!mul_ok((i128)operand[j], (i128)x[src], &p) || !add_ok(acc, p, &acc))
                    return ORC_EOVERFLOW;
            }
            if (!fits(acc, w)) return ORC_EOVERFLOW;
            out[t] = (int64_t)acc;
        }
        return ORC_OK;
    }
    case ORC_OUTER: {
        if (n_out != n_in * n_operand) return ORC_EINVAL;
        for (int64_t i = 0; i < n_in; ++i)
            for (int64_t j = 0; j < n_operand; ++j) {
                i128 v;
                if (!mul_ok((i128)x[i], (i128)operand[j], &v) || !fits(v, w)) return ORC_EOVERFLOW;
                out[i * n_operand + j] = (int64_t)v;
            }
        return ORC_OK;
    }
    default:
        return ORC_EINVAL;
    }
}

/* Selected outputs of the full linear convolution, by definition, for
 * checking very long streams at sampled positions. */
int orc_conv_at(int w, int64_t n_in, const int64_t *x, int64_t K, const int64_t *g,
                int64_t count, const int64_t *pos, int64_t *out)
{
    if (w < 2 || w > 64 || n_in < 1 || K < 1 || count < 0) return ORC_EINVAL;
    for (int64_t q = 0; q < count; ++q) {
        int64_t t = pos[q];
        if (t < 0 || t >= n_in + K - 1) return ORC_EINVAL;
        i128 v;
        if (!conv_one(x, n_in, g, K, t, &v) || !fits(v, w)) return ORC_EOVERFLOW;
        out[q] = (int64_t)v;
    }
    return ORC_OK;
}

/* ------------------------------------------------ extraction and recovery */

/* Recover all M outputs at every position from the entangled outputs of the
 * M-1 streams other than r (0 <= r < M); delta[r*n ...] is never read, and
 * may be anything. Follows eq. (16)-(19) in a 2w-bit register, with three
 * readings of the printed formulas:
 *   - eq. (16) is multiplied by (-1)^M: as printed, eq. (17)-(18) recover
 *     the right values only for even M; with the factor, M = 3 and r = 0
 *     give exactly d_temp = delta_2 - S_l{delta_1} of eq. (10).
 *   - the d-hat in eq. (18) is the one just produced by eq. (17), i.e.
 *     d-hat_{(r+M-1) mod M} (identical to the printed index when r = 0).
 *   - eq. (19) runs over 1 <= m <= M-2, so that stream (r+M-2) mod M is
 *     also recovered (for M = 3 this is the last line of eq. (10)).
 * eq. (18) divides by 2^((M-1)l) with an arithmetic shift; the value is an
 * exact multiple, which is checked (ORC_EINEXACT otherwise). */
static int extract_impl(int M, int l, int w, int64_t n, const int64_t *delta, int r,
                        int64_t *dhat, int printed_sign)
{
    if (M < 3 || l < 1 || w < 4 || w > 64 || n < 0 || r < 0 || r >= M) return ORC_EINVAL;
    if ((M - 1) * l > w) return ORC_EINVAL;
    const int W2 = 2 * w;                 /* the 2w-bit temporary register */
    const int sh = W2 - (M - 1) * l;      /* shift pair of eq. (17) */
    for (int64_t i = 0; i < n; ++i) {
        /* eq. (16) */
        i128 dtemp = 0;
        for (int m = 0; m <= M - 2; ++m) {
            int src = (r + 1 + m) % M;
            i128 term = S((i128)delta[src * n + i], (M - 2 - m) * l, W2);
            int sign_even = printed_sign ? (m % 2 == 0) : ((M + m) % 2 == 0);
            dtemp = wrap(sign_even ? dtemp + term : dtemp - term, W2);
        }
        /* eq. (17): d-hat_{(r+M-1) mod M} = S_{-sh}{S_{sh}{d_temp}} */
        int last = (r + M - 1) % M;
        i128 d_last = S(S(dtemp, sh, W2), -sh, W2);
        /* eq. (18): d-hat_r = S_{-(M-1)l}{(-1)^M (d_temp - d-hat_last)} */
        i128 diff = wrap(dtemp - d_last, W2);
        if (M % 2) diff = -diff;
        i128 d_r = S(diff, -(M - 1) * l, W2);
        if (S(d_r, (M - 1) * l, W2) != diff) return ORC_EINEXACT;
        if (!fits(d_last, w) || !fits(d_r, w)) return ORC_EOVERFLOW;
        dhat[last * n + i] = (int64_t)d_last;
        dhat[r * n + i] = (int64_t)d_r;
        /* eq. (19) for m = 1 .. M-2 */
        i128 prev = d_r;
        for (int m = 1; m <= M - 2; ++m) {
            int j = (r + m) % M;
            i128 v = (i128)delta[j * n + i] - S(prev, l, W2);
            v = wrap(v, W2);
            if (!fits(v, w)) return ORC_EOVERFLOW;
            dhat[j * n + i] = (int64_t)v;
            prev = v;
        }
    }
    return ORC_OK;
}

int orc_extract(int M, int l, int w, int64_t n, const int64_t *delta, int r, int64_t *dhat)
{
    return extract_impl(M, l, w, n, delta, r, dhat, 0);
}

/* eq. (16) exactly as printed (no (-1)^M factor). Kept only so that the
 * test suite can show that the printed sign fails for odd M -- the evidence
 * for the reading used by orc_extract. Never used to produce results. */
int orc_extract_printed_sign(int M, int l, int w, int64_t n, const int64_t *delta, int r,
                             int64_t *dhat)
{
    return extract_impl(M, l, w, n, delta, r, dhat, 1);
}

/* ---------------------------------------------------- checksum baseline */

/* eq. (4): r_n = sum_m c_{m,n}. The checksum must fit in w bits. */
int orc_checksum(int M, int w, int64_t n, const int64_t *c, int64_t *rsum)
{
    if (M < 1 || w < 2 || w > 64 || n < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        i128 s = 0;
        for (int m = 0; m < M; ++m) s += (i128)c[m * n + i];
        if (!fits(s, w)) return ORC_EOVERFLOW;
        rsum[i] = (int64_t)s;
    }
    return ORC_OK;
}

/* Recovery for the checksum method of eq. (3)-(5). The paper does not print
 * it; by linearity of op, e = r op g = sum_m d_m, so the lost output is
 * d_r = e - sum_{m != r} d_m. d[r*n ...] is never read. (For op = + the
 * checksum operand is M*g, for the same reason as footnote 3.) */
int orc_checksum_recover(int M, int w, int64_t n, const int64_t *d, const int64_t *e, int r,
                         int64_t *d_r)
{
    if (M < 1 || w < 2 || w > 64 || n < 0 || r < 0 || r >= M) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        i128 s = (i128)e[i];
        for (int m = 0; m < M; ++m)
            if (m != r) s -= (i128)d[m * n + i];
        if (!fits(s, w)) return ORC_EOVERFLOW;
        d_r[i] = (int64_t)s;
    }
    return ORC_OK;
}

/* ------------------------------------------------------ matrix product */

/* One entry of the integer matrix product D = C G (C: N x P, G: P x Q,
 * row-major): D[i][j] = sum_k C[i][k] G[k][j], exact in 128 bits. The matrix
 * product is the multiplication operator of eq. (2) applied to blocks of a
 * stream: each of the M streams is an N x P block and G the shared kernel
 * matrix (Sec. IV's GEMM case). */
static int gemm_one(const int64_t *c, const int64_t *g, int64_t P, int64_t Q, int64_t i,
                    int64_t j, i128 *out)
{
    i128 acc = 0, t;
    for (int64_t k = 0; k < P; ++k) {
        if (!mul_ok((i128)c[i * P + k], (i128)g[k * Q + j], &t) || !add_ok(acc, t, &acc))
            return 0;
    }
    *out = acc;
    return 1;
}

int orc_gemm(int w, int64_t N, int64_t P, int64_t Q, const int64_t *c, const int64_t *g,
             int64_t *out)
{
    if (w < 2 || w > 64 || N < 0 || P < 0 || Q < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < Q; ++j) {
            i128 v;
            if (!gemm_one(c, g, P, Q, i, j, &v) || !fits(v, w)) return ORC_EOVERFLOW;
            out[i * Q + j] = (int64_t)v;
        }
    return ORC_OK;
}

/* Selected entries (rows[q], cols[q]) of the same product. */
int orc_gemm_at(int w, int64_t N, int64_t P, int64_t Q, const int64_t *c, const int64_t *g,
                int64_t count, const int64_t *rows, const int64_t *cols, int64_t *out)
{
    if (w < 2 || w > 64 || N < 0 || P < 0 || Q < 0 || count < 0) return ORC_EINVAL;
    for (int64_t q = 0; q < count; ++q) {
        if (rows[q] < 0 || rows[q] >= N || cols[q] < 0 || cols[q] >= Q) return ORC_EINVAL;
        i128 v;
        if (!gemm_one(c, g, P, Q, rows[q], cols[q], &v) || !fits(v, w)) return ORC_EOVERFLOW;
        out[q] = (int64_t)v;
    }
    return ORC_OK;
}
