// Streaming kernels of libne: entanglement (eq. (14)-(15)), extraction and
// recovery (eq. (16)-(19) in the 64-bit-only form of Remark 1), the
// element-wise LSB operations and the checksum method (eq. (3)-(5)).
//
// All of these are HBM-bound: each touches every sample once, so they are
// written as coalesced 16-byte loads and stores (4 int32 or 2 int64 per
// access), one position group per lane, with a grid-stride loop over a grid
// sized to keep every CU busy. Arithmetic on 64-bit words is done in
// uint64_t so that wrap-around modulo 2^64 is defined behaviour.
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kBlock = 256;

struct alignas(16) I64x2 {
    int64_t a, b;
};

__device__ __forceinline__ int64_t entangle_word(int64_t cur, int64_t prev, int l)
{
    return (int64_t)((uint64_t)cur + ((uint64_t)prev << l));
}

inline unsigned grid_for(int64_t items, int64_t per_block = kBlock, int64_t cap = 1 << 16)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ------------------------------------------------------------ entangle

// Vector body: 4 positions per lane (one 16-byte int32 load per stream, two
// 16-byte int64 stores). The lane that owns the last, partial group of 4
// finishes it element by element. Each input is loaded once: c_{M-1} is
// kept from the first step for the last.
template <int M>
__global__ __launch_bounds__(kBlock) void k_entangle_v4(PtrsI32 c, PtrsI64 e, int64_t n, int l)
{
    const int64_t groups = (n + 3) >> 2;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < groups;
         q += (int64_t)gridDim.x * kBlock) {
        const int64_t i = q << 2;
        if (i + 4 <= n) {
            const int4 last = *reinterpret_cast<const int4 *>(c.p[M - 1] + i);
            int4 prev = last;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int4 cur = (m == M - 1) ? last : *reinterpret_cast<const int4 *>(c.p[m] + i);
                I64x2 lo{entangle_word(cur.x, prev.x, l), entangle_word(cur.y, prev.y, l)};
                I64x2 hi{entangle_word(cur.z, prev.z, l), entangle_word(cur.w, prev.w, l)};
                *reinterpret_cast<I64x2 *>(e.p[m] + i) = lo;
                *reinterpret_cast<I64x2 *>(e.p[m] + i + 2) = hi;
                prev = cur;
            }
        } else {
            for (int64_t j = i; j < n; ++j) {
#pragma unroll
                for (int m = 0; m < M; ++m)
                    e.p[m][j] = entangle_word(c.p[m][j], c.p[(m + M - 1) % M][j], l);
            }
        }
    }
}

// Any alignment: one position per lane.
template <int M>
__global__ __launch_bounds__(kBlock) void k_entangle_s(PtrsI32 c, PtrsI64 e, int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t last = c.p[M - 1][i];
        int32_t prev = last;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int32_t cur = (m == M - 1) ? last : c.p[m][i];
            e.p[m][i] = entangle_word(cur, prev, l);
            prev = cur;
        }
    }
}

// In place on int64 words: all M inputs of a position are loaded before any
// store, so every output uses original values.
template <int M>
__global__ __launch_bounds__(kBlock) void k_entangle_inplace(PtrsI64 x, int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = x.p[m][i];
#pragma unroll
        for (int m = 0; m < M; ++m) x.p[m][i] = entangle_word(v[m], v[(m + M - 1) % M], l);
    }
}

__global__ __launch_bounds__(kBlock) void k_entangle_operand(const int32_t *g, int64_t *ge,
                                                             int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        ge[i] = entangle_word(g[i], g[i], l);
}

// ------------------------------------------------------------- extract

// Recovery of one position from the M-1 available entangled outputs, in
// the rotated order in[t] = delta_{(r+1+t) mod M}, t < M-1.
//
// The paper's d_temp (eq. (16), with the (-1)^M factor that makes
// eq. (17)-(18) hold for odd M) telescopes to d_{r-1} + (-1)^M 2^{(M-1)l} d_r.
// Its low (M-1)l bits are therefore exact modulo 2^64 and, sign-extended,
// give d_{r-1} (eq. (17)) without a 2w-bit register (Remark 1). The other
// outputs follow from delta_j = d_j + 2^l d_{j-1} by walking backwards,
// d_{j-1} = (delta_j - d_j) >> l, an exact shift because delta_j - d_j is
// 2^l d_{j-1}; this replaces the 2w-bit division of eq. (18) and the
// forward chain of eq. (19) and still never touches delta_r.
// out[t] receives d_{(r+1+t) mod M}; out[M-1] is d_r.
template <int M>
__device__ __forceinline__ void recover_one(const int64_t (&in)[M - 1], int64_t (&out)[M], int l)
{
    uint64_t acc = 0;
#pragma unroll
    for (int t = 0; t < M - 1; ++t) {
        const uint64_t v = (uint64_t)in[t];
        acc = (acc << l) + (((M + t) & 1) ? (uint64_t)0 - v : v);
    }
    const int s = 64 - (M - 1) * l;  // 0 <= s < 64
    int64_t cur = ((int64_t)(acc << s)) >> s;  // d_{r-1}
    out[M - 2] = cur;
#pragma unroll
    for (int t = M - 2; t >= 0; --t) {
        cur = (int64_t)((uint64_t)in[t] - (uint64_t)cur) >> l;  // d_{r+t}
        out[t == 0 ? M - 1 : t - 1] = cur;
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_extract_v2(PtrsCI64 in, PtrsI64 out, int64_t n, int l)
{
    const int64_t pairs = (n + 1) >> 1;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < pairs;
         q += (int64_t)gridDim.x * kBlock) {
        const int64_t i = q << 1;
        if (i + 2 <= n) {
            int64_t a[M - 1], b[M - 1], oa[M], ob[M];
#pragma unroll
            for (int t = 0; t < M - 1; ++t) {
                const I64x2 v = *reinterpret_cast<const I64x2 *>(in.p[t] + i);
                a[t] = v.a;
                b[t] = v.b;
            }
            recover_one<M>(a, oa, l);
            recover_one<M>(b, ob, l);
#pragma unroll
            for (int t = 0; t < M; ++t)
                *reinterpret_cast<I64x2 *>(out.p[t] + i) = I64x2{oa[t], ob[t]};
        } else {
            int64_t a[M - 1], oa[M];
#pragma unroll
            for (int t = 0; t < M - 1; ++t) a[t] = in.p[t][i];
            recover_one<M>(a, oa, l);
#pragma unroll
            for (int t = 0; t < M; ++t) out.p[t][i] = oa[t];
        }
    }
}

// Slots 0..R-1 of a series' entangled words at source position src, from
// the int32 streams c.p[u] = stream r + u (mod M): slot t is stream r+1+t,
// c_{r+1+t} + 2^l c_{r+t}. Every stream's sample is read once, all loads
// in flight together; src < 0 gives zeros.
template <int M, int R>
__device__ __forceinline__ void entangle_slots(const PtrsI32 &c, int64_t src, int l,
                                               int64_t (&e)[R])
{
    int64_t v[M];
#pragma unroll
    for (int u = 0; u < M; ++u) v[u] = 0;
    if (src >= 0) {
#pragma unroll
        for (int u = 0; u < M; ++u) v[u] = c.p[u][src];
    }
#pragma unroll
    for (int t = 0; t < R; ++t)
        e[t] = (int64_t)((uint64_t)v[(t + 1) % M] + ((uint64_t)v[t] << l));
}

// A series' first run of element-wise operations with the entanglement on
// load (see launch_segment_entangle).
template <int M>
__global__ __launch_bounds__(kBlock) void k_segment_entangle(PtrsI32 c, Segment seg, PtrsI64 y,
                                                             int count, int64_t n, int l,
                                                             uint32_t *err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t src = i;
        if (seg.perm) {
            src = seg.p[i];
            if (src < 0 || src >= n) {
                bad = true;
                src = -1;
            }
        }
        int64_t e[M];
        entangle_slots<M, M>(c, src, l, e);
        segment_ops_all<int64_t, M>(e, seg, i);
#pragma unroll
        for (int t = 0; t < M; ++t)
            if (t < count) y.p[t][i] = e[t];
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

// Recovery fused into a series' last run of element-wise operations (see
// launch_segment_extract).
template <int M, bool ENT>
__global__ __launch_bounds__(kBlock) void k_segment_extract(PtrsCI64 in, PtrsI32 c, Segment seg,
                                                            PtrsI64 out, int64_t n, int l,
                                                            uint32_t *err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t src = i;
        if (seg.perm) {
            src = seg.p[i];
            if (src < 0 || src >= n) {
                bad = true;
                src = -1;
            }
        }
        // every stream's word first (independent loads in flight together),
        // then the run on all of them
        int64_t a[M - 1], oa[M];
#pragma unroll
        for (int t = 0; t < M - 1; ++t) a[t] = 0;
        if (ENT) {
            entangle_slots<M, M - 1>(c, src, l, a);
        } else if (src >= 0) {
            if (seg.rows > 0) {
                const int64_t *row = in.p[0] + src * seg.rows;
#pragma unroll
                for (int t = 0; t < M - 1; ++t) a[t] = row[t];
            } else {
#pragma unroll
                for (int t = 0; t < M - 1; ++t) a[t] = in.p[t][src];
            }
        }
        segment_ops_all<int64_t, M - 1>(a, seg, i);
        recover_one<M>(a, oa, l);
#pragma unroll
        for (int t = 0; t < M; ++t) out.p[t][i] = oa[t];
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_extract_s(PtrsCI64 in, PtrsI64 out, int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t a[M - 1], oa[M];
#pragma unroll
        for (int t = 0; t < M - 1; ++t) a[t] = in.p[t][i];
        recover_one<M>(a, oa, l);
#pragma unroll
        for (int t = 0; t < M; ++t) out.p[t][i] = oa[t];
    }
}

// ---------------------------------------------------- element-wise ops

template <typename T>
__device__ __forceinline__ int64_t widen(T v) { return (int64_t)v; }

// y = s * x (mod 2^64); blockIdx.y picks the stream.
template <typename Ptrs>
__global__ __launch_bounds__(kBlock) void k_scale(Ptrs x, PtrsI64 y, int64_t n, int64_t sv)
{
    const auto *xs = x.p[blockIdx.y];
    int64_t *ys = y.p[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        ys[i] = (int64_t)((uint64_t)widen(xs[i]) * (uint64_t)sv);
}

// y = x + g, or x - g with SUB (mod 2^64)
template <typename Ptrs, typename G, bool SUB = false>
__global__ __launch_bounds__(kBlock) void k_add(Ptrs x, const G *g, PtrsI64 y, int64_t n)
{
    const auto *xs = x.p[blockIdx.y];
    int64_t *ys = y.p[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const uint64_t gv = (uint64_t)widen(g[i]);
        ys[i] = (int64_t)((uint64_t)widen(xs[i]) + (SUB ? (uint64_t)0 - gv : gv));
    }
}

// y = x * g element by element (mod 2^64)
template <typename Ptrs>
__global__ __launch_bounds__(kBlock) void k_mul(Ptrs x, const int32_t *g, PtrsI64 y, int64_t n)
{
    const auto *xs = x.p[blockIdx.y];
    int64_t *ys = y.p[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        ys[i] = (int64_t)((uint64_t)widen(xs[i]) * (uint64_t)(int64_t)g[i]);
}

// y[i K + j] = x[i] g[j] (mod 2^64). Every lane owns one output index at a
// time (consecutive lanes, consecutive outputs: coalesced stores); the row
// i = idx / K and column j advance incrementally, so the loop divides only
// once per lane.
template <typename Ptrs>
__global__ __launch_bounds__(kBlock) void k_outer(Ptrs x, const int32_t *g, PtrsI64 y, int64_t n,
                                                  int64_t K)
{
    const auto *xs = x.p[blockIdx.y];
    int64_t *ys = y.p[blockIdx.y];
    const int64_t total = n * K, step = (int64_t)gridDim.x * kBlock;
    int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= total) return;
    int64_t i = idx / K, j = idx - i * K;
    const int64_t di = step / K, dj = step - di * K;
    for (; idx < total; idx += step) {
        ys[idx] = (int64_t)((uint64_t)widen(xs[i]) * (uint64_t)(int64_t)g[j]);
        i += di;
        j += dj;
        if (j >= K) {
            j -= K;
            ++i;
        }
    }
}

// y[i] = x[p[i]] (gather). An index outside [0, n) is not a permutation
// index: nothing is read for it, y[i] = 0, and NE_FLAG_PERM_INDEX is raised
// in the library's device flag word (ne_device_flags).
template <typename Ptrs>
__global__ __launch_bounds__(kBlock) void k_perm(Ptrs x, const int32_t *p, PtrsI64 y, int64_t n,
                                                 uint32_t *err)
{
    const auto *xs = x.p[blockIdx.y];
    int64_t *ys = y.p[blockIdx.y];
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t src = p[i];
        const bool ok = src >= 0 && src < n;
        bad |= !ok;
        ys[i] = ok ? widen(xs[src]) : 0;
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

__global__ __launch_bounds__(kBlock) void k_zero_first(PtrsI64 y)
{
    if (threadIdx.x == 0) y.p[blockIdx.x][0] = 0;
}

// y[0] += sum_i x[i] g[i] (mod 2^64): per-lane partial sums, a wave
// reduction with cross-lane shuffles, one LDS slot per wave, and one 64-bit
// atomic add per block. Integer addition modulo 2^64 is associative, so the
// result does not depend on the order the atomics land in.
template <typename Ptrs>
__global__ __launch_bounds__(kBlock) void k_inner(Ptrs x, const int32_t *g, PtrsI64 y, int64_t n)
{
    const auto *xs = x.p[blockIdx.y];
    uint64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        acc += (uint64_t)widen(xs[i]) * (uint64_t)(int64_t)g[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        acc += (uint64_t)__shfl_xor((unsigned long long)acc, off, 64);
    __shared__ uint64_t part[kBlock / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        atomicAdd(reinterpret_cast<unsigned long long *>(y.p[blockIdx.y]),
                  (unsigned long long)t);
    }
}

// ------------------------------------------------------ checksum method

__global__ __launch_bounds__(kBlock) void k_checksum(PtrsI32 c, int M, int64_t *r, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int64_t s = 0;
        for (int m = 0; m < M; ++m) s += c.p[m][i];
        r[i] = s;
    }
}

// d_r = e - sum of the `count` other outputs (already compacted).
__global__ __launch_bounds__(kBlock) void k_checksum_recover(PtrsCI64 d, int count,
                                                             const int64_t *e, int64_t *dr,
                                                             int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        uint64_t s = (uint64_t)e[i];
        for (int m = 0; m < count; ++m) s -= (uint64_t)d.p[m][i];
        dr[i] = (int64_t)s;
    }
}

template <int M>
void entangle_m(int l, int64_t n, const PtrsI32 &c, const PtrsI64 &e, hipStream_t s)
{
    bool vec = true;
    for (int m = 0; m < M; ++m) vec = vec && aligned16(c.p[m]) && aligned16(e.p[m]);
    if (vec)
        hipLaunchKernelGGL(k_entangle_v4<M>, dim3(grid_for((n + 3) / 4)), dim3(kBlock), 0, s, c, e,
                           n, l);
    else
        hipLaunchKernelGGL(k_entangle_s<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, c, e, n, l);
}

template <int M>
void entangle_inplace_m(int l, int64_t n, const PtrsI64 &x, hipStream_t s)
{
    hipLaunchKernelGGL(k_entangle_inplace<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, l);
}

template <int M>
void extract_m(int l, int64_t n, const PtrsCI64 &in, const PtrsI64 &out, hipStream_t s)
{
    bool vec = true;
    for (int t = 0; t < M - 1; ++t) vec = vec && aligned16(in.p[t]);
    for (int t = 0; t < M; ++t) vec = vec && aligned16(out.p[t]);
    if (vec)
        hipLaunchKernelGGL(k_extract_v2<M>, dim3(grid_for((n + 1) / 2)), dim3(kBlock), 0, s, in,
                           out, n, l);
    else
        hipLaunchKernelGGL(k_extract_s<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, in, out, n, l);
}

// Dispatch a runtime M in [3, kMaxM] to a template instantiation.
#define NE_DISPATCH_M(M, FN, ...)                                                          \
    switch (M) {                                                                           \
    case 3: FN<3>(__VA_ARGS__); break;   case 4: FN<4>(__VA_ARGS__); break;                \
    case 5: FN<5>(__VA_ARGS__); break;   case 6: FN<6>(__VA_ARGS__); break;                \
    case 7: FN<7>(__VA_ARGS__); break;   case 8: FN<8>(__VA_ARGS__); break;                \
    case 9: FN<9>(__VA_ARGS__); break;   case 10: FN<10>(__VA_ARGS__); break;              \
    case 11: FN<11>(__VA_ARGS__); break; case 12: FN<12>(__VA_ARGS__); break;              \
    case 13: FN<13>(__VA_ARGS__); break; case 14: FN<14>(__VA_ARGS__); break;              \
    case 15: FN<15>(__VA_ARGS__); break; case 16: FN<16>(__VA_ARGS__); break;              \
    case 17: FN<17>(__VA_ARGS__); break; case 18: FN<18>(__VA_ARGS__); break;              \
    case 19: FN<19>(__VA_ARGS__); break; case 20: FN<20>(__VA_ARGS__); break;              \
    case 21: FN<21>(__VA_ARGS__); break; case 22: FN<22>(__VA_ARGS__); break;              \
    case 23: FN<23>(__VA_ARGS__); break; case 24: FN<24>(__VA_ARGS__); break;              \
    case 25: FN<25>(__VA_ARGS__); break; case 26: FN<26>(__VA_ARGS__); break;              \
    case 27: FN<27>(__VA_ARGS__); break; case 28: FN<28>(__VA_ARGS__); break;              \
    case 29: FN<29>(__VA_ARGS__); break; case 30: FN<30>(__VA_ARGS__); break;              \
    case 31: FN<31>(__VA_ARGS__); break; case 32: FN<32>(__VA_ARGS__); break;              \
    default: break;                                                                        \
    }

}  // namespace

void launch_entangle(int M, int l, int64_t n, const PtrsI32 &c, const PtrsI64 &eps, hipStream_t s)
{
    NE_DISPATCH_M(M, entangle_m, l, n, c, eps, s);
}

void launch_entangle_inplace(int M, int l, int64_t n, const PtrsI64 &x, hipStream_t s)
{
    NE_DISPATCH_M(M, entangle_inplace_m, l, n, x, s);
}

namespace {
template <int M>
void segment_extract_m(int l, int64_t n, bool entangle, const PtrsCI64 &in, const PtrsI32 &c,
                       const Segment &seg, const PtrsI64 &out, uint32_t *err, hipStream_t s)
{
    if (entangle)
        hipLaunchKernelGGL((k_segment_extract<M, true>), dim3(grid_for(n)), dim3(kBlock), 0, s, in,
                           c, seg, out, n, l, err);
    else
        hipLaunchKernelGGL((k_segment_extract<M, false>), dim3(grid_for(n)), dim3(kBlock), 0, s,
                           in, c, seg, out, n, l, err);
}

template <int M>
void segment_entangle_m(int l, int64_t n, int count, const PtrsI32 &c, const Segment &seg,
                        const PtrsI64 &y, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL(k_segment_entangle<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, c, seg, y,
                       count, n, l, err);
}
}  // namespace

void launch_segment_extract(int M, int l, int64_t n, bool entangle, const PtrsCI64 &in,
                            const PtrsI32 &c, const Segment &seg, const PtrsI64 &out,
                            uint32_t *err, hipStream_t s)
{
    NE_DISPATCH_M(M, segment_extract_m, l, n, entangle, in, c, seg, out, err, s);
}

void launch_segment_entangle(int M, int l, int64_t n, int count, const PtrsI32 &c,
                             const Segment &seg, const PtrsI64 &y, uint32_t *err, hipStream_t s)
{
    NE_DISPATCH_M(M, segment_entangle_m, l, n, count, c, seg, y, err, s);
}

void launch_entangle_operand(int l, int64_t n, const int32_t *g, int64_t *g_ent, hipStream_t s)
{
    hipLaunchKernelGGL(k_entangle_operand, dim3(grid_for(n)), dim3(kBlock), 0, s, g, g_ent, n, l);
}

void launch_extract(int M, int l, int64_t n, const PtrsCI64 &in, const PtrsI64 &out, hipStream_t s)
{
    NE_DISPATCH_M(M, extract_m, l, n, in, out, s);
}

void launch_scale_i64(int count, int64_t n, const PtrsCI64 &x, int64_t sv, const PtrsI64 &y,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_scale<PtrsCI64>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0,
                       s, x, y, n, sv);
}

void launch_add_i64(int count, int64_t n, const PtrsCI64 &x, const int64_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_add<PtrsCI64, int64_t>), dim3(grid_for(n, kBlock, 4096), count),
                       dim3(kBlock), 0, s, x, g, y, n);
}

void launch_sub_i64(int count, int64_t n, const PtrsCI64 &x, const int64_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_add<PtrsCI64, int64_t, true>), dim3(grid_for(n, kBlock, 4096), count),
                       dim3(kBlock), 0, s, x, g, y, n);
}

void launch_mul_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_mul<PtrsCI64>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0, s,
                       x, g, y, n);
}

void launch_outer_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                      const PtrsI64 &y, hipStream_t s)
{
    hipLaunchKernelGGL(k_outer<PtrsCI64>, dim3(grid_for(n * K, kBlock, 4096), count), dim3(kBlock),
                       0, s, x, g, y, n, K);
}

void launch_perm_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *p, const PtrsI64 &y,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_perm<PtrsCI64>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0,
                       s, x, p, y, n, device_flag_word());
}

void launch_inner_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, const PtrsI64 &y,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_first, dim3(count), dim3(64), 0, s, y);
    hipLaunchKernelGGL(k_inner<PtrsCI64>, dim3(grid_for(n, kBlock * 8, 1024), count),
                       dim3(kBlock), 0, s, x, g, y, n);
}

void launch_scale_i32(int count, int64_t n, const PtrsI32 &x, int64_t sv, const PtrsI64 &y,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_scale<PtrsI32>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0,
                       s, x, y, n, sv);
}

void launch_add_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_add<PtrsI32, int32_t>), dim3(grid_for(n, kBlock, 4096), count),
                       dim3(kBlock), 0, s, x, g, y, n);
}

void launch_sub_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_add<PtrsI32, int32_t, true>), dim3(grid_for(n, kBlock, 4096), count),
                       dim3(kBlock), 0, s, x, g, y, n);
}

void launch_mul_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_mul<PtrsI32>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0, s,
                       x, g, y, n);
}

void launch_outer_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, int64_t K,
                      const PtrsI64 &y, hipStream_t s)
{
    hipLaunchKernelGGL(k_outer<PtrsI32>, dim3(grid_for(n * K, kBlock, 4096), count), dim3(kBlock),
                       0, s, x, g, y, n, K);
}

void launch_perm_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *p, const PtrsI64 &y,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_perm<PtrsI32>, dim3(grid_for(n, kBlock, 4096), count), dim3(kBlock), 0,
                       s, x, p, y, n, device_flag_word());
}

void launch_inner_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_first, dim3(count), dim3(64), 0, s, y);
    hipLaunchKernelGGL(k_inner<PtrsI32>, dim3(grid_for(n, kBlock * 8, 1024), count), dim3(kBlock),
                       0, s, x, g, y, n);
}

void launch_checksum(int M, int64_t n, const PtrsI32 &c, int64_t *rsum, hipStream_t s)
{
    hipLaunchKernelGGL(k_checksum, dim3(grid_for(n)), dim3(kBlock), 0, s, c, M, rsum, n);
}

void launch_checksum_recover(int count, int64_t n, const PtrsCI64 &d, const int64_t *e,
                             int64_t *d_r, hipStream_t s)
{
    hipLaunchKernelGGL(k_checksum_recover, dim3(grid_for(n)), dim3(kBlock), 0, s, d, count, e, d_r,
                       n);
}

}  // namespace ne
