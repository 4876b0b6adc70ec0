// Series of LSB operations on entangled streams (ne_chain_*): the shape and
// range bookkeeping of the series (host) and its execution as one launch
// per stage over ping-pong buffers in the caller's workspace (or, for
// ne_chain_apply_noalloc, in a fixed device buffer of the library's own).
// A stage is one operation on the per-step kernels of ne_lsb_apply, or a
// run of element-wise operations (led, optionally, by a permutation) fused
// into one pass over the entangled words.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "ne_internal.h"

using namespace ne;

namespace {

constexpr int32_t kMaxChainOps = 64;
constexpr size_t kWsAlign = 256;

inline size_t align_up(size_t x) { return (x + kWsAlign - 1) & ~(kWsAlign - 1); }

// Output length of one operation on n_in samples, or -1 for a shape error
// (-2: unknown operation).
int64_t stage_out(const ne_chain_op &o, int64_t n_in)
{
    switch (o.op) {
    case NE_OP_CONV:
    case NE_OP_XCORR:
        if (o.n_operand < 1) return -1;
        return n_in == 0 ? 0 : n_in + o.n_operand - 1;
    case NE_OP_CIRC:
        if (o.n_operand < 1) return -1;
        return n_in;
    case NE_OP_OUTER:
        if (o.n_operand < 0 || (o.n_operand > 0 && n_in > INT64_MAX / 8 / o.n_operand)) return -1;
        return n_in * o.n_operand;
    case NE_OP_SCALE: return n_in;
    case NE_OP_ADD:
    case NE_OP_SUB:
    case NE_OP_MUL:
    case NE_OP_PERM:
        if (o.n_operand != n_in) return -1;
        if (o.op == NE_OP_PERM && n_in > INT32_MAX) return -1;
        return n_in;
    case NE_OP_INNER:
        if (o.n_operand != n_in) return -1;
        return 1;
    default: return -2;
    }
}

bool uses_operand_bits(int32_t op) { return op != NE_OP_SCALE && op != NE_OP_PERM; }

// Walks the series: the output length of every stage, and the longest
// intermediate (every stage but the last).
ne_status walk(int64_t n_in, const ne_chain_op *ops, int32_t n_ops, int64_t *n_out,
               int64_t *longest)
{
    if (n_in < 0 || !ops || n_ops < 1 || n_ops > kMaxChainOps) return NE_EINVAL;
    int64_t n = n_in, lg = 0;
    for (int32_t i = 0; i < n_ops; ++i) {
        const ne_chain_op &o = ops[i];
        const int64_t m = stage_out(o, n);
        if (m == -2) return NE_EUNSUP;
        if (m < 0) return NE_EINVAL;
        if (uses_operand_bits(o.op) && (o.operand_bits < 1 || o.operand_bits > 32))
            return NE_EINVAL;
        if (i + 1 < n_ops) lg = std::max(lg, m);
        n = m;
    }
    if (n_out) *n_out = n;
    if (longest) *longest = lg;
    return NE_OK;
}

// The range bookkeeping of a series in w-bit words (groups of up to max_m
// streams).
ne_status check_w(int32_t M, int32_t w, int32_t max_m, int32_t in_bits, int64_t n_in,
                  const ne_chain_op *ops, int32_t n_ops, int64_t *n_out, int64_t *bound)
{
    if (M < 3 || M > max_m || in_bits < 1 || in_bits > 32) return NE_EINVAL;
    const ne_status st = walk(n_in, ops, n_ops, n_out, nullptr);
    if (st != NE_OK) return st;
    int64_t D = 0;
    if (ne_params(M, w, nullptr, nullptr, &D) != NE_OK) return NE_ERANGE;
    // Worst-case |d| after each stage, in 128 bits; products saturate, so an
    // absurd operand length cannot wrap below D.
    using u128 = unsigned __int128;
    const auto mul = [](u128 a, u128 b) { return (b != 0 && a > ~(u128)0 / b) ? ~(u128)0 : a * b; };
    u128 B = (u128)1 << (in_bits - 1);
    if (B > (u128)D) return NE_ERANGE;
    int64_t n = n_in;
    for (int32_t i = 0; i < n_ops; ++i) {
        const ne_chain_op &o = ops[i];
        const u128 G = uses_operand_bits(o.op) ? (u128)1 << (o.operand_bits - 1) : 0;
        switch (o.op) {
        case NE_OP_CONV:
        case NE_OP_CIRC:
        case NE_OP_XCORR: B = mul(mul(B, G), (u128)o.n_operand); break;
        case NE_OP_MUL:
        case NE_OP_OUTER: B = mul(B, G); break;
        case NE_OP_SCALE: {
            const u128 s = o.scalar < 0 ? (u128)0 - (u128)(__int128)o.scalar : (u128)o.scalar;
            if (s > ((u128)1 << 62)) return NE_ERANGE;
            B = mul(B, s);
            break;
        }
        case NE_OP_ADD:
        case NE_OP_SUB: B = B + G; break;
        case NE_OP_INNER: B = mul(mul(B, G), (u128)std::max<int64_t>(n, 1)); break;
        case NE_OP_PERM: break;
        }
        if (B > (u128)D) return NE_ERANGE;
        n = stage_out(o, n);
    }
    if (bound) *bound = (int64_t)B;
    return NE_OK;
}

ne_status workspace_w(int32_t M, int64_t n_in, const ne_chain_op *ops, int32_t n_ops,
                      size_t word, size_t *bytes)
{
    if (M < 1 || M > kMaxM || !bytes) return NE_EINVAL;
    int64_t longest = 0;
    const ne_status st = walk(n_in, ops, n_ops, nullptr, &longest);
    if (st != NE_OK) return st;
    *bytes = n_ops > 1 ? 2 * (size_t)M * align_up((size_t)longest * word) : 0;
    return NE_OK;
}

// Intermediates of ne_chain_apply_noalloc: a fixed buffer in device memory,
// one copy on every device that loads the library, held until the process
// ends. On the host, `scratch` only stands in for the device array: kernels
// and copies take the per-device address that hipGetSymbolAddress returns
// (scratch_address), never the array's name.
static __device__ __align__(256) unsigned char scratch[NE_CHAIN_SCRATCH_BYTES];

// The address of `scratch` on the calling thread's current device, looked
// up once per device with that device current and kept; NULL with *st set
// on a HIP error.
unsigned char *scratch_address(ne_status *st)
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static unsigned char *addr[kDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *st = hip_fail(e);
        return nullptr;
    }
    if (dev < 0 || dev >= kDevices) {
        *st = NE_EUNSUP;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *st = hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        addr[dev] = (unsigned char *)p;
    }
    return addr[dev];
}

// ------------------------------------------------ fused element-wise runs

// A run of consecutive element-wise operations of a series (scale, add, sub,
// mul), optionally led by a permutation, applied in one pass over the
// entangled words: out[i] = op_k( ... op_1(in[p[i]] or in[i]) ...).
constexpr int kMaxSegmentOps = 8;
struct SegmentOp {
    int32_t op;
    int32_t pad_;
    const void *g;  // NE_OP_ADD / NE_OP_SUB: words of the stream width; NE_OP_MUL: int32
    int64_t s;      // NE_OP_SCALE
};
struct Segment {
    int32_t nops;
    int32_t perm;          // 1: gather at p[i] first
    const int32_t *p;
    SegmentOp ops[kMaxSegmentOps];
};

inline bool elementwise(int32_t op)
{
    return op == NE_OP_SCALE || op == NE_OP_ADD || op == NE_OP_SUB || op == NE_OP_MUL;
}

// blockIdx.y picks the stream; W is the word (int64_t or int32_t), arithmetic
// wraps modulo 2^(8 sizeof W). A permutation index outside [0, n) reads
// nothing (the word is 0) and raises NE_FLAG_PERM_INDEX.
template <typename W, typename In, typename Out>
__global__ __launch_bounds__(256) void k_segment(In x, Out y, int64_t n, Segment seg,
                                                 uint32_t *err)
{
    using U = typename std::make_unsigned<W>::type;
    const W *xs = x.p[blockIdx.y];
    W *ys = y.p[blockIdx.y];
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        U v;
        if (seg.perm) {
            const int64_t src = seg.p[i];
            const bool ok = src >= 0 && src < n;
            bad |= !ok;
            v = ok ? (U)xs[src] : (U)0;
        } else {
            v = (U)xs[i];
        }
        for (int k = 0; k < seg.nops; ++k) {
            const SegmentOp &o = seg.ops[k];
            switch (o.op) {
            case NE_OP_SCALE: v = v * (U)o.s; break;
            case NE_OP_ADD: v = v + (U)((const W *)o.g)[i]; break;
            case NE_OP_SUB: v = v - (U)((const W *)o.g)[i]; break;
            default: v = v * (U)(W)((const int32_t *)o.g)[i]; break;  // NE_OP_MUL
            }
        }
        ys[i] = (W)v;
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

template <typename W, typename In, typename Out>
void launch_segment(int count, int64_t n, const In &x, const Out &y, const Segment &seg,
                    hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL((k_segment<W, In, Out>), dim3((unsigned)g, count), dim3(256), 0, s, x, y, n,
                       seg, device_flag_word());
}

// Word-width traits of the series' execution: the stream tables and the
// launch of one operation.
struct Words64 {
    using W = int64_t;
    using In = PtrsCI64;
    using Out = PtrsI64;
    static ne_status launch(const ne_chain_op &o, int count, int64_t n, const In &cur,
                            const Out &dst, int64_t m, hipStream_t s)
    {
        switch (o.op) {
        case NE_OP_CONV:
            launch_conv_i64(count, n, cur, (const int32_t *)o.operand, o.n_operand, dst, s);
            break;
        case NE_OP_SCALE: launch_scale_i64(count, n, cur, o.scalar, dst, s); break;
        case NE_OP_ADD: launch_add_i64(count, n, cur, (const int64_t *)o.operand, dst, s); break;
        case NE_OP_INNER:
            launch_inner_i64(count, n, cur, (const int32_t *)o.operand, dst, s);
            break;
        case NE_OP_PERM:
            launch_perm_i64(count, n, cur, (const int32_t *)o.operand, dst, s);
            break;
        case NE_OP_SUB: launch_sub_i64(count, n, cur, (const int64_t *)o.operand, dst, s); break;
        case NE_OP_MUL: launch_mul_i64(count, n, cur, (const int32_t *)o.operand, dst, s); break;
        case NE_OP_CIRC:
            launch_conv_i64(count, n, cur, (const int32_t *)o.operand, o.n_operand, dst, s,
                            kConvCircular);
            break;
        case NE_OP_XCORR:
            launch_conv_i64(count, n, cur, (const int32_t *)o.operand, o.n_operand, dst, s,
                            kConvXcorr);
            break;
        case NE_OP_OUTER:
            launch_outer_i64(count, n, cur, (const int32_t *)o.operand, o.n_operand, dst, s);
            break;
        }
        return launch_status();
    }
    static ne_status segment(const Segment &seg, int count, int64_t n, const In &cur,
                             const Out &dst, hipStream_t s)
    {
        launch_segment<W>(count, n, cur, dst, seg, s);
        return launch_status();
    }
};

struct Words32 {
    using W = int32_t;
    using In = PtrsI32;
    using Out = PtrsW32;
    static ne_status launch(const ne_chain_op &o, int count, int64_t n, const In &cur,
                            const Out &dst, int64_t m, hipStream_t s)
    {
        launch_op32(o.op, count, n, cur, (const int32_t *)o.operand, o.n_operand, o.scalar, dst,
                    m, s);
        return launch_status();
    }
    static ne_status segment(const Segment &seg, int count, int64_t n, const In &cur,
                             const Out &dst, hipStream_t s)
    {
        launch_segment<W>(count, n, cur, dst, seg, s);
        return launch_status();
    }
};

template <typename T>
ne_status apply_w(int32_t M, int64_t n_in, const typename T::W *const *eps,
                  const ne_chain_op *ops, int32_t n_ops, typename T::W *const *delta,
                  int64_t n_out, uint32_t stream_mask, void *workspace, size_t workspace_bytes,
                  ne_stream stream, bool use_scratch = false)
{
    using W = typename T::W;
    if (M < 1 || M > kMaxM || !eps || !delta) return NE_EINVAL;
    int64_t want = 0, longest = 0;
    ne_status st = walk(n_in, ops, n_ops, &want, &longest);
    if (st != NE_OK) return st;
    if (n_out != want) return NE_EINVAL;
    const size_t plane = align_up((size_t)longest * sizeof(W));
    const bool need_ws = n_ops > 1 && plane > 0;
    if (need_ws && use_scratch) {
        if (2 * (size_t)M * plane > NE_CHAIN_SCRATCH_BYTES) return NE_ESCRATCH;
    } else if (need_ws) {
        if (!workspace || workspace_bytes < 2 * (size_t)M * plane) return NE_EINVAL;
        if ((uintptr_t)workspace % kWsAlign) return NE_EINVAL;
    }
    for (int32_t i = 0; i < n_ops; ++i) {
        const ne_chain_op &o = ops[i];
        const bool needs = o.op == NE_OP_CONV || (o.op != NE_OP_SCALE && o.n_operand > 0);
        if (needs && !o.operand) return NE_EINVAL;
    }
    if (M < 32) stream_mask &= (1u << M) - 1u;
    // The computed streams, compacted; stage i reads `cur` and writes the
    // workspace buffer (i & 1), or delta for the last stage.
    typename T::In cur{};
    typename T::Out fin{};
    int count = 0;
    for (int m = 0; m < M; ++m) {
        if (!((stream_mask >> m) & 1u)) continue;
        if ((!eps[m] && n_in > 0) || (!delta[m] && n_out > 0)) return NE_EINVAL;
        cur.p[count] = eps[m];
        fin.p[count] = delta[m];
        ++count;
    }
    if (count == 0) return NE_OK;
    if (need_ws && use_scratch) {
        // every argument has been checked: only now is the device touched
        ne_status sst = NE_OK;
        workspace = scratch_address(&sst);
        if (!workspace) return sst;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char *ws = (unsigned char *)workspace;
    int64_t n = n_in;
    // Stages: a run of element-wise operations (led, optionally, by a
    // permutation) is one pass; every other operation is a pass of its own.
    // Stage k writes workspace buffer (k & 1), the last one delta.
    int stage = 0;
    for (int32_t i = 0; i < n_ops;) {
        const ne_chain_op &o = ops[i];
        int32_t j = i + 1;  // the stage is ops [i, j)
        if (o.op == NE_OP_PERM || elementwise(o.op))
            while (j < n_ops && j - i < kMaxSegmentOps && elementwise(ops[j].op)) ++j;
        int64_t m = n;
        for (int32_t k = i; k < j; ++k) m = stage_out(ops[k], m);
        typename T::Out dst{};
        if (j == n_ops) {
            dst = fin;
        } else {
            for (int t = 0; t < count; ++t)
                dst.p[t] = (W *)(ws + ((size_t)(stage & 1) * M + t) * plane);
        }
        if (m > 0) {
            if (j - i == 1 && !(o.op == NE_OP_PERM || elementwise(o.op))) {
                st = T::launch(o, count, n, cur, dst, m, s);
            } else {
                Segment seg{};
                seg.perm = o.op == NE_OP_PERM;
                seg.p = seg.perm ? (const int32_t *)o.operand : nullptr;
                for (int32_t k = i + seg.perm; k < j; ++k) {
                    SegmentOp &so = seg.ops[seg.nops++];
                    so.op = ops[k].op;
                    so.g = ops[k].operand;
                    so.s = ops[k].scalar;
                }
                st = T::segment(seg, count, n, cur, dst, s);
            }
            if (st != NE_OK) return st;
        }
        for (int t = 0; t < count; ++t) cur.p[t] = dst.p[t];
        n = m;
        i = j;
        ++stage;
    }
    return NE_OK;
}

}  // namespace

extern "C" {

ne_status ne_chain_check(int32_t M, int32_t in_bits, int64_t n_in, const ne_chain_op *ops,
                         int32_t n_ops, int64_t *n_out, int64_t *bound)
{
    return check_w(M, 64, kMaxM, in_bits, n_in, ops, n_ops, n_out, bound);
}

ne_status ne_chain_workspace_size(int32_t M, int64_t n_in, const ne_chain_op *ops, int32_t n_ops,
                                  size_t *bytes)
{
    return workspace_w(M, n_in, ops, n_ops, sizeof(int64_t), bytes);
}

ne_status ne_chain_apply(int32_t M, int64_t n_in, const int64_t *const *eps,
                         const ne_chain_op *ops, int32_t n_ops, int64_t *const *delta,
                         int64_t n_out, uint32_t stream_mask, void *workspace,
                         size_t workspace_bytes, ne_stream stream)
{
    return apply_w<Words64>(M, n_in, eps, ops, n_ops, delta, n_out, stream_mask, workspace,
                            workspace_bytes, stream);
}

ne_status ne_chain_apply_noalloc(int32_t M, int64_t n_in, const int64_t *const *eps,
                                 const ne_chain_op *ops, int32_t n_ops, int64_t *const *delta,
                                 int64_t n_out, uint32_t stream_mask, ne_stream stream)
{
    return apply_w<Words64>(M, n_in, eps, ops, n_ops, delta, n_out, stream_mask, nullptr, 0,
                            stream, true);
}

ne_status ne_chain_check32(int32_t M, int32_t in_bits, int64_t n_in, const ne_chain_op *ops,
                           int32_t n_ops, int64_t *n_out, int64_t *bound)
{
    return check_w(M, 32, NE_MAX_M32, in_bits, n_in, ops, n_ops, n_out, bound);
}

ne_status ne_chain_workspace_size32(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                    int32_t n_ops, size_t *bytes)
{
    return workspace_w(M, n_in, ops, n_ops, sizeof(int32_t), bytes);
}

ne_status ne_chain_apply32(int32_t M, int64_t n_in, const int32_t *const *eps,
                           const ne_chain_op *ops, int32_t n_ops, int32_t *const *delta,
                           int64_t n_out, uint32_t stream_mask, void *workspace,
                           size_t workspace_bytes, ne_stream stream)
{
    return apply_w<Words32>(M, n_in, eps, ops, n_ops, delta, n_out, stream_mask, workspace,
                            workspace_bytes, stream);
}


}  // extern "C"
