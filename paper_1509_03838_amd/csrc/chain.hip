// Series of LSB operations on entangled streams (ne_chain_*): the shape and
// range bookkeeping of the series (host) and its execution as one launch
// per stage over ping-pong buffers in the caller's workspace (or, for
// ne_chain_apply_noalloc, in a fixed device buffer of the library's own).
// A stage is one operation on the per-step kernels of ne_lsb_apply, or a
// run of element-wise operations (led, optionally, by a permutation) fused
// into one pass over the entangled words. ne_chain_run adds the
// entanglement and the recovery, fused into the first and the last run of
// element-wise operations where the series begins or ends with one.
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
    const W *xs = x.p[blockIdx.y];
    W *ys = y.p[blockIdx.y];
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        W v = 0;
        if (seg.perm) {
            const int64_t src = seg.p[i];
            const bool ok = src >= 0 && src < n;
            bad |= !ok;
            if (ok) v = xs[src];
        } else {
            v = xs[i];
        }
        ys[i] = segment_ops<W>(v, seg, i);
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

// A run led by a permutation whose input rows hold the R streams' words of
// each position (Segment::rows = R): every lane gathers all R words of its
// source position from one row, so a random position costs one fetch of R
// words rather than R fetches of one.
template <typename W, typename Out, int R>
__global__ __launch_bounds__(256) void k_segment_rows(const W *x, Out y, int64_t n, Segment seg,
                                                      uint32_t *err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        int64_t src = i;
        if (seg.perm) {
            src = seg.p[i];
            if (src < 0 || src >= n) {
                bad = true;
                src = -1;
            }
        }
        W v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = src >= 0 ? x[src * R + t] : 0;
        segment_ops_all<W, R>(v, seg, i);
#pragma unroll
        for (int t = 0; t < R; ++t) y.p[t][i] = v[t];
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

// Streams a convolution may interleave into rows for the gather after it.
constexpr int kMaxRows = 8;

template <typename W, typename Out>
void launch_segment_rows(int count, int64_t n, const W *x, const Out &y, const Segment &seg,
                         hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    const dim3 grid((unsigned)g), block(256);
    uint32_t *err = device_flag_word();
#define NE_ROWS_CASE(R)                                                                   \
    hipLaunchKernelGGL((k_segment_rows<W, Out, R>), grid, block, 0, s, x, y, n, seg, err)
    switch (count) {  // 1..kMaxRows: rows_after admits no more
    case 1: NE_ROWS_CASE(1); break;
    case 2: NE_ROWS_CASE(2); break;
    case 3: NE_ROWS_CASE(3); break;
    case 4: NE_ROWS_CASE(4); break;
    case 5: NE_ROWS_CASE(5); break;
    case 6: NE_ROWS_CASE(6); break;
    case 7: NE_ROWS_CASE(7); break;
    default: NE_ROWS_CASE(8); break;
    }
#undef NE_ROWS_CASE
}

template <typename W, typename In, typename Out>
void launch_segment(int count, int64_t n, const In &x, const Out &y, const Segment &seg,
                    hipStream_t s)
{
    if (seg.rows > 0) {
        launch_segment_rows<W>(count, n, x.p[0], y, seg, s);
        return;
    }
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL((k_segment<W, In, Out>), dim3((unsigned)g, count), dim3(256), 0, s, x, y, n,
                       seg, device_flag_word());
}

// Word-width traits of the series' execution: the stream tables and the
// launch of one operation.
inline bool conv_kind(int32_t op)
{
    return op == NE_OP_CONV || op == NE_OP_CIRC || op == NE_OP_XCORR;
}

struct Words64 {
    using W = int64_t;
    using In = PtrsCI64;
    using Out = PtrsI64;
    static constexpr bool kRows = true;  // convolutions can write rows
    static constexpr int kWidth = 64;
    static constexpr int kGroupMax = kMaxM;
    static void seg_entangle(int M, int l, int64_t n, int count, const PtrsI32 &c,
                             const Segment &seg, const Out &y, uint32_t *err, hipStream_t s)
    {
        launch_segment_entangle(M, l, n, count, c, seg, y, err, s);
    }
    static void seg_extract(int M, int l, int64_t n, bool entangle, const In &in,
                            const PtrsI32 &c, const Segment &seg, const Out &out, uint32_t *err,
                            hipStream_t s)
    {
        launch_segment_extract(M, l, n, entangle, in, c, seg, out, err, s);
    }
    static void extract(int M, int l, int64_t n, const In &in, const Out &out, hipStream_t s)
    {
        launch_extract(M, l, n, in, out, s);
    }
    static ne_status conv_rows(const ne_chain_op &o, int count, int64_t n, const In &cur,
                               int64_t *rows, hipStream_t s)
    {
        const int kind = o.op == NE_OP_CIRC ? kConvCircular
                                            : (o.op == NE_OP_XCORR ? kConvXcorr : kConvLinear);
        launch_conv_i64_rows(count, n, cur, (const int32_t *)o.operand, o.n_operand, rows, s, kind);
        return launch_status();
    }
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
    static constexpr bool kRows = true;  // convolutions can write rows
    static constexpr int kWidth = 32;
    static constexpr int kGroupMax = NE_MAX_M32;
    static void seg_entangle(int M, int l, int64_t n, int count, const PtrsI32 &c,
                             const Segment &seg, const Out &y, uint32_t *err, hipStream_t s)
    {
        launch_segment_entangle32(M, l, n, count, c, seg, y, err, s);
    }
    static void seg_extract(int M, int l, int64_t n, bool entangle, const In &in,
                            const PtrsI32 &c, const Segment &seg, const Out &out, uint32_t *err,
                            hipStream_t s)
    {
        launch_segment_extract32(M, l, n, entangle, in, c, seg, out, err, s);
    }
    static void extract(int M, int l, int64_t n, const In &in, const Out &out, hipStream_t s)
    {
        launch_extract32(M, l, n, in, out, s);
    }
    static ne_status conv_rows(const ne_chain_op &o, int count, int64_t n, const In &cur,
                               int32_t *rows, hipStream_t s)
    {
        const int64_t n_out = o.op == NE_OP_CIRC ? n : n + o.n_operand - 1;
        launch_conv32_rows(o.op, count, n, cur, (const int32_t *)o.operand, o.n_operand, n_out,
                           rows, s);
        return launch_status();
    }
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

// The stages of a series: a run of element-wise operations (led, optionally,
// by a permutation; at most kMaxSegmentOps) is one stage, every other
// operation a stage of its own. Stage k is ops [i, j) on n_in samples.
struct Stage {
    int32_t i, j;
    bool seg;
    int64_t n_in, n_out;
};

int split_stages(const ne_chain_op *ops, int32_t n_ops, int64_t n_in, Stage *out)
{
    int ns = 0;
    int64_t n = n_in;
    for (int32_t i = 0; i < n_ops;) {
        const ne_chain_op &o = ops[i];
        int32_t j = i + 1;
        const bool seg = o.op == NE_OP_PERM || elementwise(o.op);
        if (seg)
            while (j < n_ops && j - i < kMaxSegmentOps && elementwise(ops[j].op)) ++j;
        int64_t m = n;
        for (int32_t k = i; k < j; ++k) m = stage_out(ops[k], m);
        out[ns++] = Stage{i, j, seg, n, m};
        n = m;
        i = j;
    }
    return ns;
}

// Stage k, a convolution whose output a permutation-led run gathers next,
// writes that output as rows of its `count` streams (kMaxRows at most).
bool rows_after(const ne_chain_op *ops, const Stage *st, int ns, int k, int count)
{
    return k + 1 < ns && !st[k].seg && conv_kind(ops[st[k].i].op) && st[k + 1].seg &&
           ops[st[k + 1].i].op == NE_OP_PERM && count <= kMaxRows;
}

Segment make_segment(const ne_chain_op *ops, const Stage &g, int rows = 0)
{
    Segment seg{};
    seg.perm = ops[g.i].op == NE_OP_PERM;
    seg.p = seg.perm ? (const int32_t *)ops[g.i].operand : nullptr;
    seg.rows = rows;
    for (int32_t k = g.i + seg.perm; k < g.j; ++k) {
        SegmentOp &so = seg.ops[seg.nops++];
        so.op = ops[k].op;
        so.g = ops[k].operand;
        so.s = ops[k].scalar;
    }
    return seg;
}

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
    // Stage k writes workspace buffer (k & 1), the last one delta; a
    // convolution before a permutation-led run writes rows there (the
    // buffer's M planes hold count rows of the longest stage).
    Stage stages[kMaxChainOps];
    const int ns = split_stages(ops, n_ops, n_in, stages);
    int rows_in = 0;  // > 0: the current input is in rows of that many words
    for (int k = 0; k < ns; ++k) {
        const Stage &g = stages[k];
        const bool to_rows = T::kRows && rows_after(ops, stages, ns, k, count);
        typename T::Out dst{};
        if (k == ns - 1) {
            dst = fin;
        } else {
            for (int t = 0; t < count; ++t)
                dst.p[t] = (W *)(ws + ((size_t)(k & 1) * M + t) * plane);
        }
        if (g.n_out > 0) {
            if (g.seg)
                st = T::segment(make_segment(ops, g, rows_in), count, g.n_in, cur, dst, s);
            else if (to_rows)
                st = T::conv_rows(ops[g.i], count, g.n_in, cur, dst.p[0], s);
            else
                st = T::launch(ops[g.i], count, g.n_in, cur, dst, g.n_out, s);
            if (st != NE_OK) return st;
        }
        rows_in = to_rows ? count : 0;
        for (int t = 0; t < count; ++t) cur.p[t] = dst.p[t];
    }
    return NE_OK;
}

// ------------------------------------------------ the whole method on a series

// Workspace of ne_chain_run: two buffers of M planes of words of `word`
// bytes, each as long as the longest intermediate -- every stage's output
// but the last, and the entangled inputs when the first stage cannot
// entangle them on load -- or nothing when the series is one run of
// element-wise operations.
ne_status run_workspace(int32_t M, int64_t n_in, const ne_chain_op *ops, int32_t n_ops,
                        size_t word, size_t *bytes)
{
    int64_t longest = 0;
    const ne_status st = walk(n_in, ops, n_ops, nullptr, &longest);
    if (st != NE_OK) return st;
    Stage stages[kMaxChainOps];
    const int ns = split_stages(ops, n_ops, n_in, stages);
    if (!stages[0].seg) longest = std::max(longest, n_in);
    const bool need = ns > 1 || !stages[0].seg;
    *bytes = need ? 2 * (size_t)M * align_up((size_t)longest * word) : 0;
    return NE_OK;
}

// Entangle, run the series on every computed stream, extract and recover,
// in words of T's width. Computed streams in slot order: slot t is stream
// (r + 1 + t) mod M, the order recovery reads (slot M - 1, stream r, only
// when nothing was lost).
template <typename T>
ne_status chain_run(int32_t M, int64_t n_in, const int32_t *const *c, const ne_chain_op *ops,
                    int32_t n_ops, int32_t lost, typename T::W *const *dhat, int64_t n_out,
                    void *workspace, size_t workspace_bytes, ne_stream stream)
{
    using W = typename T::W;
    if (M < 3 || M > T::kGroupMax || !c || !dhat) return NE_EINVAL;
    if (lost < -1 || lost >= M) return NE_EFAILIDX;
    int64_t want = 0;
    ne_status st = walk(n_in, ops, n_ops, &want, nullptr);
    if (st != NE_OK) return st;
    if (n_out != want) return NE_EINVAL;
    for (int32_t i = 0; i < n_ops; ++i) {
        const ne_chain_op &o = ops[i];
        const bool needs = o.op == NE_OP_CONV || (o.op != NE_OP_SCALE && o.n_operand > 0);
        if (needs && !o.operand) return NE_EINVAL;
    }
    for (int m = 0; m < M; ++m)
        if ((!c[m] && n_in > 0) || (!dhat[m] && n_out > 0)) return NE_EINVAL;
    int32_t l = 0;
    if (ne_params(M, T::kWidth, &l, nullptr, nullptr) != NE_OK) return NE_ERANGE;
    size_t need = 0;
    st = run_workspace(M, n_in, ops, n_ops, sizeof(W), &need);
    if (st != NE_OK) return st;
    if (need > 0 && (!workspace || workspace_bytes < need || (uintptr_t)workspace % kWsAlign))
        return NE_EINVAL;
    if (n_out == 0) return NE_OK;

    Stage stages[kMaxChainOps];
    const int ns = split_stages(ops, n_ops, n_in, stages);
    const int r = lost >= 0 ? lost : 0;
    const int count = lost >= 0 ? M - 1 : M;  // computed streams
    PtrsI32 cr{};  // the int32 streams from r on: slot t entangles cr[t + 1] with cr[t]
    typename T::Out out{};
    for (int t = 0; t < M; ++t) {
        cr.p[t] = c[(r + t) % M];
        out.p[t] = dhat[(r + 1 + t) % M];
    }
    hipStream_t s = (hipStream_t)stream;
    uint32_t *err = device_flag_word();
    const size_t plane = need / (2 * (size_t)M);
    unsigned char *ws = (unsigned char *)workspace;
    auto buffer = [&](int b) {
        typename T::Out p{};
        for (int t = 0; t < count; ++t) p.p[t] = (W *)(ws + ((size_t)b * M + t) * plane);
        return p;
    };
    typename T::In cur{};
    if (!stages[0].seg) {
        // a first stage that cannot entangle on load: the entangled words
        // first, into buffer 1 (stage 0 writes buffer 0)
        const typename T::Out e = buffer(1);
        T::seg_entangle(M, l, n_in, count, cr, Segment{}, e, err, s);
        for (int t = 0; t < count; ++t) cur.p[t] = e.p[t];
    }
    int rows_in = 0;  // > 0: the current input is in rows of that many words
    for (int k = 0; k < ns; ++k) {
        const Stage &g = stages[k];
        const bool first = k == 0, last = k == ns - 1;
        if (last && g.seg) {
            // the last run with the recovery (and, as the only stage, the
            // entanglement) in the same pass
            T::seg_extract(M, l, g.n_in, first, cur, cr, make_segment(ops, g, rows_in), out, err,
                           s);
            return launch_status();
        }
        const bool to_rows = T::kRows && rows_after(ops, stages, ns, k, count);
        typename T::Out dst = last ? out : buffer(k & 1);
        if (g.n_out > 0) {
            if (first && g.seg)
                T::seg_entangle(M, l, g.n_in, count, cr, make_segment(ops, g), dst, err, s);
            else if (g.seg)
                launch_segment<W>(count, g.n_in, cur, dst, make_segment(ops, g, rows_in), s);
            else if (to_rows)
                T::conv_rows(ops[g.i], count, g.n_in, cur, dst.p[0], s);
            else
                T::launch(ops[g.i], count, g.n_in, cur, dst, g.n_out, s);
            st = launch_status();
            if (st != NE_OK) return st;
        }
        rows_in = to_rows ? count : 0;
        for (int t = 0; t < count; ++t) cur.p[t] = dst.p[t];
    }
    // the last stage wrote the computed streams' words into dhat: recover in place
    typename T::In in{};
    for (int t = 0; t < M - 1; ++t) in.p[t] = out.p[t];
    T::extract(M, l, n_out, in, out, s);
    return launch_status();
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

ne_status ne_chain_run_workspace_size(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                      int32_t n_ops, size_t *bytes)
{
    if (M < 3 || M > kMaxM || !bytes) return NE_EINVAL;
    return run_workspace(M, n_in, ops, n_ops, sizeof(int64_t), bytes);
}

ne_status ne_chain_run(int32_t M, int64_t n_in, const int32_t *const *c, const ne_chain_op *ops,
                       int32_t n_ops, int32_t lost, int64_t *const *dhat, int64_t n_out,
                       void *workspace, size_t workspace_bytes, ne_stream stream)
{
    return chain_run<Words64>(M, n_in, c, ops, n_ops, lost, dhat, n_out, workspace,
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

ne_status ne_chain_run_workspace_size32(int32_t M, int64_t n_in, const ne_chain_op *ops,
                                        int32_t n_ops, size_t *bytes)
{
    if (M < 3 || M > NE_MAX_M32 || !bytes) return NE_EINVAL;
    return run_workspace(M, n_in, ops, n_ops, sizeof(int32_t), bytes);
}

ne_status ne_chain_run32(int32_t M, int64_t n_in, const int32_t *const *c, const ne_chain_op *ops,
                         int32_t n_ops, int32_t lost, int32_t *const *dhat, int64_t n_out,
                         void *workspace, size_t workspace_bytes, ne_stream stream)
{
    return chain_run<Words32>(M, n_in, c, ops, n_ops, lost, dhat, n_out, workspace,
                              workspace_bytes, stream);
}


}  // extern "C"
