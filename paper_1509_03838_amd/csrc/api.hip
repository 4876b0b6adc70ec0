// C-ABI of libne (include/ne.h): argument validation, stream-mask
// compaction, the stream rotation used by recovery, and dispatch to the
// kernels. Nothing here allocates memory; only ne_device_flags (documented
// as synchronous) synchronises the device.
#include <string.h>

#include <mutex>
#include <type_traits>

#include "ne_internal.h"

namespace ne {

static thread_local int32_t g_last_hip_error = 0;

ne_status hip_fail(hipError_t e)
{
    g_last_hip_error = (int32_t)e;
    return NE_EHIP;
}

ne_status launch_status()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? NE_OK : hip_fail(e);
}

ne_status check_op_shape(int32_t op, int64_t n_in, const void *operand, int64_t n_operand,
                         int64_t n_out)
{
    if (n_in < 0 || n_operand < 0 || n_out < 0) return NE_EINVAL;
    switch (op) {
    case NE_OP_CONV:
    case NE_OP_XCORR:
        if (n_operand < 1 || !operand) return NE_EINVAL;
        if (n_out != (n_in == 0 ? 0 : n_in + n_operand - 1)) return NE_EINVAL;
        return NE_OK;
    case NE_OP_CIRC:
        if (n_operand < 1 || !operand || n_out != n_in) return NE_EINVAL;
        return NE_OK;
    case NE_OP_OUTER:
        if (n_operand > 0 && n_in > INT64_MAX / n_operand) return NE_EUNSUP;
        if (n_out != n_in * n_operand) return NE_EINVAL;
        if (n_operand > 0 && !operand) return NE_EINVAL;
        return NE_OK;
    case NE_OP_SCALE:
        return n_out == n_in ? NE_OK : NE_EINVAL;
    case NE_OP_ADD:
    case NE_OP_SUB:
    case NE_OP_MUL:
    case NE_OP_PERM:
        if (n_operand != n_in || n_out != n_in) return NE_EINVAL;
        if (n_in > 0 && !operand) return NE_EINVAL;
        if (op == NE_OP_PERM && n_in > INT32_MAX) return NE_EUNSUP;
        return NE_OK;
    case NE_OP_INNER:
        if (n_operand != n_in || n_out != 1) return NE_EINVAL;
        if (n_in > 0 && !operand) return NE_EINVAL;
        return NE_OK;
    default:
        return NE_EUNSUP;
    }
}

// The per-step kernels' device flag word: one copy per device (each device
// that loads the library's code object holds its own), found by symbol
// lookup with that device current and cached per device.
static __device__ uint32_t g_device_flags;

uint32_t *device_flag_word()
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static uint32_t *addr[kDevices];
    static bool done[kDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!done[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_device_flags)) == hipSuccess)
            addr[dev] = (uint32_t *)p;
        else
            (void)hipGetLastError();
        done[dev] = true;
    }
    return addr[dev];
}

}  // namespace ne

using namespace ne;

namespace {

inline bool bad_m(int32_t M, int32_t lo) { return M < lo || M > kMaxM; }

// Copies the streams whose mask bit is set into a compacted table.
template <typename In, typename Tab>
int compact(int32_t M, In const *const *src, uint32_t mask, Tab &dst, bool &null_seen)
{
    int count = 0;
    null_seen = false;
    for (int m = 0; m < M; ++m) {
        if (!((mask >> m) & 1u)) continue;
        if (!src[m]) null_seen = true;
        using P = std::remove_reference_t<decltype(dst.p[0])>;
        dst.p[count++] = const_cast<P>(src[m]);
    }
    return count;
}

}  // namespace

extern "C" {

const char *ne_strerror(ne_status s)
{
    switch (s) {
    case NE_OK: return "ok";
    case NE_EINVAL: return "invalid argument";
    case NE_ERANGE: return "no admissible shift/headroom for this group size and word width";
    case NE_EFAILIDX: return "failed-stream index out of range";
    case NE_EUNSUP: return "operation or shape not supported";
    case NE_EHIP: return "HIP runtime error";
    case NE_ENOMEM: return "device allocation failed";
    case NE_ESCRATCH: return "needs more than the library's fixed scratch buffer";
    case NE_ELATE: return "more than one stream missed the deadline";
    default: return "unknown status";
    }
}

int32_t ne_last_hip_error(void) { return g_last_hip_error; }

int32_t ne_version(void) { return 10000 * 0 + 100 * 2 + 0; }

ne_status ne_device_flags(uint32_t *flags, int32_t clear)
{
    if (!flags) return NE_EINVAL;
    uint32_t *w = device_flag_word();
    if (!w) return hip_fail(hipErrorInvalidSymbol);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(flags, w, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && clear) {
        const uint32_t z = 0;
        e = hipMemcpy(w, &z, sizeof(uint32_t), hipMemcpyHostToDevice);
    }
    return e == hipSuccess ? NE_OK : hip_fail(e);
}

// Closed form of the Table I rule: the output bit-width (M-2)l + k with
// k = w - (M-1)l is w - l, which decreases in l, while k <= l needs
// l >= w/M; so l = ceil(w/M) unless that leaves k < 0, in which case no l
// makes k = w - (M-1)l admissible, k <= l binds, the width is (M-1)l, and
// l = floor(w/M), k = l.
ne_status ne_params(int32_t M, int32_t w, int32_t *l_out, int32_t *k_out, int64_t *dmax)
{
    if (M < 3 || M > kMaxM || w < 8 || w > 64) return NE_EINVAL;
    if (!l_out && !k_out && !dmax) return NE_EINVAL;
    int l = (w + M - 1) / M;
    int k = w - (M - 1) * l;
    if (k < 0) {
        l = w / M;
        k = l;
    }
    if (l < 2) return NE_ERANGE;  // l = 1 makes eq. (13) empty
    __int128 D;
    if (M == 3)
        D = ((__int128)1 << (l + k - 1)) - ((__int128)1 << l);          // eq. (11)
    else
        D = ((__int128)1 << ((M - 3) * l + k)) * (((__int128)1 << (l - 1)) - 1);  // eq. (13)
    if (D < 1) return NE_ERANGE;
    if (l_out) *l_out = l;
    if (k_out) *k_out = k;
    if (dmax) *dmax = (int64_t)D;
    return NE_OK;
}

ne_status ne_entangle(int32_t M, int32_t l, int64_t n, const int32_t *const *c,
                      int64_t *const *eps, ne_stream stream)
{
    if (bad_m(M, 3) || l < 1 || l > 63 || n < 0 || !c || !eps) return NE_EINVAL;
    if (n == 0) return NE_OK;
    PtrsI32 pc{};
    PtrsI64 pe{};
    for (int m = 0; m < M; ++m) {
        if (!c[m] || !eps[m]) return NE_EINVAL;
        pc.p[m] = c[m];
        pe.p[m] = eps[m];
    }
    launch_entangle(M, l, n, pc, pe, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_entangle_inplace(int32_t M, int32_t l, int64_t n, int64_t *const *x,
                              ne_stream stream)
{
    if (bad_m(M, 3) || l < 1 || l > 63 || n < 0 || !x) return NE_EINVAL;
    if (n == 0) return NE_OK;
    PtrsI64 px{};
    for (int m = 0; m < M; ++m) {
        if (!x[m]) return NE_EINVAL;
        px.p[m] = x[m];
    }
    launch_entangle_inplace(M, l, n, px, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_entangle_operand(int32_t l, int64_t n, const int32_t *g, int64_t *g_ent,
                              ne_stream stream)
{
    if (l < 1 || l > 63 || n < 0) return NE_EINVAL;
    if (n == 0) return NE_OK;
    if (!g || !g_ent) return NE_EINVAL;
    launch_entangle_operand(l, n, g, g_ent, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_lsb_apply(int32_t op, int32_t M, int64_t n_in, const int64_t *const *eps,
                       const void *operand, int64_t n_operand, int64_t scalar,
                       int64_t *const *delta, int64_t n_out, uint32_t stream_mask,
                       ne_stream stream)
{
    if (bad_m(M, 1) || !eps || !delta) return NE_EINVAL;
    ne_status st = check_op_shape(op, n_in, operand, n_operand, n_out);
    if (st != NE_OK) return st;
    if (M < 32) stream_mask &= (1u << M) - 1u;
    PtrsCI64 px{};
    PtrsI64 py{};
    bool nx = false, ny = false;
    const int count = compact(M, eps, stream_mask, px, nx);
    compact(M, delta, stream_mask, py, ny);
    if ((nx && n_in > 0) || (ny && n_out > 0)) return NE_EINVAL;
    if (count == 0 || n_out == 0) return NE_OK;
    hipStream_t s = (hipStream_t)stream;
    switch (op) {
    case NE_OP_CONV:
        launch_conv_i64(count, n_in, px, (const int32_t *)operand, n_operand, py, s);
        break;
    case NE_OP_SCALE: launch_scale_i64(count, n_in, px, scalar, py, s); break;
    case NE_OP_ADD: launch_add_i64(count, n_in, px, (const int64_t *)operand, py, s); break;
    case NE_OP_INNER: launch_inner_i64(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_PERM: launch_perm_i64(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_SUB: launch_sub_i64(count, n_in, px, (const int64_t *)operand, py, s); break;
    case NE_OP_MUL: launch_mul_i64(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_CIRC:
        launch_conv_i64(count, n_in, px, (const int32_t *)operand, n_operand, py, s, kConvCircular);
        break;
    case NE_OP_XCORR:
        launch_conv_i64(count, n_in, px, (const int32_t *)operand, n_operand, py, s, kConvXcorr);
        break;
    case NE_OP_OUTER:
        launch_outer_i64(count, n_in, px, (const int32_t *)operand, n_operand, py, s);
        break;
    }
    return launch_status();
}

ne_status ne_extract_recover(int32_t M, int32_t l, int64_t n_out, const int64_t *const *delta,
                             int32_t r, int64_t *const *dhat, ne_stream stream)
{
    if (bad_m(M, 3) || l < 1 || l > 63 || (M - 1) * l > 64 || n_out < 0 || !delta || !dhat)
        return NE_EINVAL;
    if (r < -1 || r >= M) return NE_EFAILIDX;
    if (n_out == 0) return NE_OK;
    if (r < 0) r = 0;
    // Rotate so that the kernel sees delta_{r+1}, ..., delta_{r+M-1} and
    // writes d_{r+1}, ..., d_{r+M-1}, d_r with compile-time indices.
    PtrsCI64 in{};
    PtrsI64 out{};
    for (int t = 0; t < M - 1; ++t) {
        const int j = (r + 1 + t) % M;
        if (!delta[j]) return NE_EINVAL;
        in.p[t] = delta[j];
    }
    for (int t = 0; t < M; ++t) {
        const int j = (r + 1 + t) % M;
        if (!dhat[j]) return NE_EINVAL;
        out.p[t] = dhat[j];
    }
    launch_extract(M, l, n_out, in, out, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_plain_apply(int32_t op, int32_t n_streams, int64_t n_in, const int32_t *const *c,
                         const void *operand, int64_t n_operand, int64_t scalar,
                         int64_t *const *d, int64_t n_out, ne_stream stream)
{
    if (bad_m(n_streams, 1) || !c || !d) return NE_EINVAL;
    ne_status st = check_op_shape(op, n_in, operand, n_operand, n_out);
    if (st != NE_OK) return st;
    const uint32_t all = n_streams < 32 ? (1u << n_streams) - 1u : 0xffffffffu;
    PtrsI32 px{};
    PtrsI64 py{};
    bool nx = false, ny = false;
    const int count = compact(n_streams, c, all, px, nx);
    compact(n_streams, d, all, py, ny);
    if ((nx && n_in > 0) || (ny && n_out > 0)) return NE_EINVAL;
    if (n_out == 0) return NE_OK;
    hipStream_t s = (hipStream_t)stream;
    switch (op) {
    case NE_OP_CONV:
        launch_conv_i32(count, n_in, px, (const int32_t *)operand, n_operand, py, s);
        break;
    case NE_OP_SCALE: launch_scale_i32(count, n_in, px, scalar, py, s); break;
    case NE_OP_ADD: launch_add_i32(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_INNER: launch_inner_i32(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_PERM: launch_perm_i32(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_SUB: launch_sub_i32(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_MUL: launch_mul_i32(count, n_in, px, (const int32_t *)operand, py, s); break;
    case NE_OP_CIRC:
        launch_conv_i32(count, n_in, px, (const int32_t *)operand, n_operand, py, s, kConvCircular);
        break;
    case NE_OP_XCORR:
        launch_conv_i32(count, n_in, px, (const int32_t *)operand, n_operand, py, s, kConvXcorr);
        break;
    case NE_OP_OUTER:
        launch_outer_i32(count, n_in, px, (const int32_t *)operand, n_operand, py, s);
        break;
    }
    return launch_status();
}

ne_status ne_checksum(int32_t M, int64_t n, const int32_t *const *c, int64_t *rsum,
                      ne_stream stream)
{
    if (bad_m(M, 1) || n < 0 || !c) return NE_EINVAL;
    if (n == 0) return NE_OK;
    if (!rsum) return NE_EINVAL;
    PtrsI32 pc{};
    for (int m = 0; m < M; ++m) {
        if (!c[m]) return NE_EINVAL;
        pc.p[m] = c[m];
    }
    launch_checksum(M, n, pc, rsum, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_checksum_recover(int32_t M, int64_t n_out, const int64_t *const *d,
                              const int64_t *e, int32_t r, int64_t *d_r, ne_stream stream)
{
    if (bad_m(M, 1) || n_out < 0 || !d) return NE_EINVAL;
    if (r < 0 || r >= M) return NE_EFAILIDX;
    if (n_out == 0) return NE_OK;
    if (!e || !d_r) return NE_EINVAL;
    PtrsCI64 pd{};
    int count = 0;
    for (int m = 0; m < M; ++m) {
        if (m == r) continue;
        if (!d[m]) return NE_EINVAL;
        pd.p[count++] = d[m];
    }
    launch_checksum_recover(count, n_out, pd, e, d_r, (hipStream_t)stream);
    return launch_status();
}

}  // extern "C"
