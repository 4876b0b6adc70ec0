// The method in 32-bit entangled words: the paper's practical
// instantiation (Sec. III-B with Table I's w = 32 column; l = 11, k = 10
// for M = 3). Entanglement, every LSB operation, and extraction with
// recovery work on int32 words modulo 2^32, so every word that crosses HBM
// is half as wide as in the 64-bit path; the price is the smaller output
// range (|d| <= D of ne_params(M, 32): 1,046,528 for M = 3).
//
// Kernels: entanglement and extraction move 4 positions per lane with
// 16-byte accesses; the element-wise operations likewise; the
// convolution-like operations are the direct VALU convolution (one 32-bit
// multiply-add per tap and output, accumulated modulo 2^32); the inner
// product reduces per block and adds with one 32-bit atomic. Arithmetic is
// done in uint32_t so that wrap-around is defined behaviour.
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t items, int64_t per_block = kBlock, int64_t cap = 1 << 16)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

__device__ __forceinline__ int32_t ent32(int32_t cur, int32_t prev, int l)
{
    return (int32_t)((uint32_t)cur + ((uint32_t)prev << l));
}

__device__ __forceinline__ int4 ld4(const int32_t *p) { return *reinterpret_cast<const int4 *>(p); }
__device__ __forceinline__ void st4(int32_t *p, int4 v) { *reinterpret_cast<int4 *>(p) = v; }

// ------------------------------------------------------------ entangle

// eps_m = c_m + 2^l c_{m-1} (mod 2^32), 4 positions per lane; the lane that
// owns the last, partial group finishes it one position at a time.
template <int M>
__global__ __launch_bounds__(kBlock) void k_entangle32_v4(PtrsI32 c, PtrsW32 e, int64_t n, int l)
{
    const int64_t groups = (n + 3) >> 2;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < groups;
         q += (int64_t)gridDim.x * kBlock) {
        const int64_t i = q << 2;
        if (i + 4 <= n) {
            const int4 last = ld4(c.p[M - 1] + i);
            int4 prev = last;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int4 cur = (m == M - 1) ? last : ld4(c.p[m] + i);
                st4(e.p[m] + i, int4{ent32(cur.x, prev.x, l), ent32(cur.y, prev.y, l),
                                     ent32(cur.z, prev.z, l), ent32(cur.w, prev.w, l)});
                prev = cur;
            }
        } else {
            for (int64_t j = i; j < n; ++j) {
#pragma unroll
                for (int m = 0; m < M; ++m)
                    e.p[m][j] = ent32(c.p[m][j], c.p[(m + M - 1) % M][j], l);
            }
        }
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_entangle32_s(PtrsI32 c, PtrsW32 e, int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int m = 0; m < M; ++m) e.p[m][i] = ent32(c.p[m][i], c.p[(m + M - 1) % M][i], l);
    }
}

__global__ __launch_bounds__(kBlock) void k_entangle_operand32(const int32_t *g, int32_t *ge,
                                                               int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        ge[i] = ent32(g[i], g[i], l);
}

// ------------------------------------------------------------- extract

// Recovery of one position in 32-bit words; in[t] = delta_{(r+1+t) mod M}.
// The sign-corrected d_temp of eq. (16) telescopes to
// d_{r-1} + (-1)^M 2^{(M-1)l} d_r, so its low (M-1)l <= 32 bits, computed
// modulo 2^32 and sign-extended, are d_{r-1} (eq. (17)); the others follow
// backwards from delta_j = d_j + 2^l d_{j-1}: d_{j-1} = (delta_j - d_j) >> l,
// exact because |2^l d| < 2^31 within the range of eq. (11)/(13). delta_r is
// never used. out[t] receives d_{(r+1+t) mod M}; out[M-1] is d_r.
template <int M>
__device__ __forceinline__ void recover32(const int32_t (&in)[M - 1], int32_t (&out)[M], int l)
{
    uint32_t acc = 0;
#pragma unroll
    for (int t = 0; t < M - 1; ++t) {
        const uint32_t v = (uint32_t)in[t];
        acc = (acc << l) + (((M + t) & 1) ? 0u - v : v);
    }
    const int s = 32 - (M - 1) * l;  // 0 <= s < 32
    int32_t cur = ((int32_t)(acc << s)) >> s;  // d_{r-1}
    out[M - 2] = cur;
#pragma unroll
    for (int t = M - 2; t >= 0; --t) {
        cur = (int32_t)((uint32_t)in[t] - (uint32_t)cur) >> l;  // d_{r+t}
        out[t == 0 ? M - 1 : t - 1] = cur;
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_extract32_v4(PtrsI32 in, PtrsW32 out, int64_t n, int l)
{
    const int64_t groups = (n + 3) >> 2;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < groups;
         q += (int64_t)gridDim.x * kBlock) {
        const int64_t i = q << 2;
        if (i + 4 <= n) {
            int32_t a[4][M - 1], o[4][M];
#pragma unroll
            for (int t = 0; t < M - 1; ++t) {
                const int4 v = ld4(in.p[t] + i);
                a[0][t] = v.x;
                a[1][t] = v.y;
                a[2][t] = v.z;
                a[3][t] = v.w;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) recover32<M>(a[u], o[u], l);
#pragma unroll
            for (int t = 0; t < M; ++t) st4(out.p[t] + i, int4{o[0][t], o[1][t], o[2][t], o[3][t]});
        } else {
            for (int64_t j = i; j < n; ++j) {
                int32_t a[M - 1], o[M];
#pragma unroll
                for (int t = 0; t < M - 1; ++t) a[t] = in.p[t][j];
                recover32<M>(a, o, l);
#pragma unroll
                for (int t = 0; t < M; ++t) out.p[t][j] = o[t];
            }
        }
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_extract32_s(PtrsI32 in, PtrsW32 out, int64_t n, int l)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int32_t a[M - 1], o[M];
#pragma unroll
        for (int t = 0; t < M - 1; ++t) a[t] = in.p[t][i];
        recover32<M>(a, o, l);
#pragma unroll
        for (int t = 0; t < M; ++t) out.p[t][i] = o[t];
    }
}

// ---------------------------------------------------- element-wise ops

enum MapOp { kMapScale, kMapAdd, kMapSub, kMapMul };

template <int OP>
__device__ __forceinline__ int32_t map1(int32_t x, int32_t g, uint32_t sv)
{
    const uint32_t ux = (uint32_t)x, ug = (uint32_t)g;
    if (OP == kMapScale) return (int32_t)(ux * sv);
    if (OP == kMapAdd) return (int32_t)(ux + ug);
    if (OP == kMapSub) return (int32_t)(ux - ug);
    return (int32_t)(ux * ug);
}

// y = x op g (or s x) on one stream per blockIdx.y, modulo 2^32. VEC: every
// pointer is 16-byte aligned, 4 positions per lane.
template <int OP, bool VEC>
__global__ __launch_bounds__(kBlock) void k_map32(PtrsI32 x, const int32_t *g, PtrsW32 y,
                                                  int64_t n, uint32_t sv)
{
    const int32_t *xs = x.p[blockIdx.y];
    int32_t *ys = y.p[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (VEC) {
        const int64_t groups = (n + 3) >> 2;
        for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < groups; q += stride) {
            const int64_t i = q << 2;
            if (i + 4 <= n) {
                const int4 a = ld4(xs + i);
                const int4 b = OP == kMapScale ? int4{0, 0, 0, 0} : ld4(g + i);
                st4(ys + i, int4{map1<OP>(a.x, b.x, sv), map1<OP>(a.y, b.y, sv),
                                 map1<OP>(a.z, b.z, sv), map1<OP>(a.w, b.w, sv)});
            } else {
                for (int64_t j = i; j < n; ++j)
                    ys[j] = map1<OP>(xs[j], OP == kMapScale ? 0 : g[j], sv);
            }
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
            ys[i] = map1<OP>(xs[i], OP == kMapScale ? 0 : g[i], sv);
    }
}

// y[i] = x[p[i]]; an index outside [0, n) reads nothing, gives y[i] = 0 and
// raises NE_FLAG_PERM_INDEX in the library's device flag word.
__global__ __launch_bounds__(kBlock) void k_perm32(PtrsI32 x, const int32_t *p, PtrsW32 y,
                                                   int64_t n, uint32_t *err)
{
    const int32_t *xs = x.p[blockIdx.y];
    int32_t *ys = y.p[blockIdx.y];
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t src = p[i];
        const bool ok = src >= 0 && src < n;
        bad |= !ok;
        ys[i] = ok ? xs[src] : 0;
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

// y[i K + j] = x[i] g[j] (mod 2^32); one output per lane, (i, j) advanced
// incrementally so each lane divides once.
__global__ __launch_bounds__(kBlock) void k_outer32(PtrsI32 x, const int32_t *g, PtrsW32 y,
                                                    int64_t n, int64_t K)
{
    const int32_t *xs = x.p[blockIdx.y];
    int32_t *ys = y.p[blockIdx.y];
    const int64_t total = n * K, step = (int64_t)gridDim.x * kBlock;
    int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= total) return;
    int64_t i = idx / K, j = idx - i * K;
    const int64_t di = step / K, dj = step - di * K;
    for (; idx < total; idx += step) {
        ys[idx] = (int32_t)((uint32_t)xs[i] * (uint32_t)g[j]);
        i += di;
        j += dj;
        if (j >= K) {
            j -= K;
            ++i;
        }
    }
}

__global__ __launch_bounds__(64) void k_zero_first32(PtrsW32 y)
{
    if (threadIdx.x == 0) y.p[blockIdx.x][0] = 0;
}

// y[0] += sum_i x[i] g[i] (mod 2^32): per-lane sums, a wave reduction, one
// LDS slot per wave and one 32-bit atomic per block; addition modulo 2^32
// is associative, so the order the atomics land in does not matter.
__global__ __launch_bounds__(kBlock) void k_inner32(PtrsI32 x, const int32_t *g, PtrsW32 y,
                                                    int64_t n)
{
    const int32_t *xs = x.p[blockIdx.y];
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        acc += (uint32_t)xs[i] * (uint32_t)g[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += (uint32_t)__shfl_xor((int)acc, off, 64);
    __shared__ uint32_t part[kBlock / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        atomicAdd(reinterpret_cast<unsigned int *>(y.p[blockIdx.y]), t);
    }
}

// ---------------------------------------------------- convolution-like

// y[t] = sum_{j<K} g[j] x[t-j] (mod 2^32): a block owns kTile outputs; per
// chunk of up to kKC taps it stages the window (zero outside [0, n), or
// wrapped modulo n for the circular kind) and the taps (reversed for the
// cross-correlation) in LDS; each lane accumulates kQ outputs kBlock apart
// (consecutive lanes read consecutive LDS words, the tap is a broadcast).
constexpr int kQ = 4;
constexpr int kTile = kBlock * kQ;
constexpr int kKC = 1024;

struct ConvArgs32 {
    PtrsI32 x;
    PtrsW32 y;
    const int32_t *g;
    int64_t n, K, n_out;
    int32_t kind;
    int32_t rows;  // 0: stream blockIdx.y's outputs to plane y.p[blockIdx.y]; > 0: to rows of
                   // that many words at y.p[0] (stream t's output i at [i * rows + t])
};

__global__ __launch_bounds__(kBlock) void k_conv32(ConvArgs32 a)
{
    __shared__ int32_t sx[kTile + kKC];
    __shared__ int32_t sg[kKC];
    const int tid = threadIdx.x;
    const int32_t *x = a.x.p[blockIdx.y];
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    uint32_t acc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = 0;
    for (int64_t j0 = 0; j0 < a.K; j0 += kKC) {
        const int kc = (int)((a.K - j0) < kKC ? (a.K - j0) : kKC);
        const int64_t wbase = t0 - j0 - (kc - 1);
        const int wlen = kTile + kc - 1;
        __syncthreads();
        for (int w = tid; w < wlen; w += kBlock) {
            int64_t idx = wbase + w;
            int32_t v = 0;
            if (a.kind == kConvCircular) {
                idx %= a.n;
                v = x[idx < 0 ? idx + a.n : idx];
            } else if (idx >= 0 && idx < a.n) {
                v = x[idx];
            }
            sx[w] = v;
        }
        for (int j = tid; j < kc; j += kBlock)
            sg[j] = a.g[a.kind == kConvXcorr ? a.K - 1 - (j0 + j) : j0 + j];
        __syncthreads();
        for (int j = 0; j < kc; ++j) {
            const uint32_t gj = (uint32_t)sg[j];
            const int wb = tid + kc - 1 - j;
#pragma unroll
            for (int q = 0; q < kQ; ++q) acc[q] += (uint32_t)sx[wb + q * kBlock] * gj;
        }
    }
    int32_t *y = a.rows ? a.y.p[0] + blockIdx.y : a.y.p[blockIdx.y];
    const int64_t stride = a.rows ? a.rows : 1;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int64_t t = t0 + q * kBlock + tid;
        if (t < a.n_out) y[t * stride] = (int32_t)acc[q];
    }
}

// ------------------------------------------------------------- launchers

template <int M>
void entangle32_m(int l, int64_t n, const PtrsI32 &c, const PtrsW32 &e, hipStream_t s)
{
    bool vec = true;
    for (int m = 0; m < M; ++m) vec = vec && aligned16(c.p[m]) && aligned16(e.p[m]);
    if (vec)
        hipLaunchKernelGGL(k_entangle32_v4<M>, dim3(grid_for((n + 3) / 4)), dim3(kBlock), 0, s, c,
                           e, n, l);
    else
        hipLaunchKernelGGL(k_entangle32_s<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, c, e, n, l);
}

template <int M>
void extract32_m(int l, int64_t n, const PtrsI32 &in, const PtrsW32 &out, hipStream_t s)
{
    bool vec = true;
    for (int t = 0; t < M - 1; ++t) vec = vec && aligned16(in.p[t]);
    for (int t = 0; t < M; ++t) vec = vec && aligned16(out.p[t]);
    if (vec)
        hipLaunchKernelGGL(k_extract32_v4<M>, dim3(grid_for((n + 3) / 4)), dim3(kBlock), 0, s, in,
                           out, n, l);
    else
        hipLaunchKernelGGL(k_extract32_s<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, in, out, n, l);
}

#define NE_DISPATCH_M32(M, FN, ...)                                                        \
    switch (M) {                                                                           \
    case 3: FN<3>(__VA_ARGS__); break;   case 4: FN<4>(__VA_ARGS__); break;                \
    case 5: FN<5>(__VA_ARGS__); break;   case 6: FN<6>(__VA_ARGS__); break;                \
    case 7: FN<7>(__VA_ARGS__); break;   case 8: FN<8>(__VA_ARGS__); break;                \
    case 9: FN<9>(__VA_ARGS__); break;   case 10: FN<10>(__VA_ARGS__); break;              \
    case 11: FN<11>(__VA_ARGS__); break; case 12: FN<12>(__VA_ARGS__); break;              \
    case 13: FN<13>(__VA_ARGS__); break; case 14: FN<14>(__VA_ARGS__); break;              \
    case 15: FN<15>(__VA_ARGS__); break; case 16: FN<16>(__VA_ARGS__); break;              \
    case 17: FN<17>(__VA_ARGS__); break;                                                   \
    default: break;                                                                        \
    }

template <int OP>
void map32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsW32 &y,
           uint32_t sv, hipStream_t s)
{
    bool vec = OP == kMapScale || aligned16(g);
    for (int t = 0; t < count; ++t) vec = vec && aligned16(x.p[t]) && aligned16(y.p[t]);
    const dim3 grid(grid_for((n + 3) / 4, kBlock, 4096), count);
    if (vec)
        hipLaunchKernelGGL((k_map32<OP, true>), grid, dim3(kBlock), 0, s, x, g, y, n, sv);
    else
        hipLaunchKernelGGL((k_map32<OP, false>), dim3(grid_for(n, kBlock, 4096), count),
                           dim3(kBlock), 0, s, x, g, y, n, sv);
}

// ------------------------------------------ series in one call (w = 32)

// Slots 0..R-1 of a series' 32-bit entangled words at source position src
// from the int32 streams c.p[u] = stream r + u (mod M): slot t is
// c_{r+1+t} + 2^l c_{r+t} (mod 2^32), each stream read once; src < 0 gives
// zeros.
template <int M, int R>
__device__ __forceinline__ void entangle_slots32(const PtrsI32 &c, int64_t src, int l,
                                                 int32_t (&e)[R])
{
    int32_t v[M];
#pragma unroll
    for (int u = 0; u < M; ++u) v[u] = 0;
    if (src >= 0) {
#pragma unroll
        for (int u = 0; u < M; ++u) v[u] = c.p[u][src];
    }
#pragma unroll
    for (int t = 0; t < R; ++t) e[t] = ent32(v[(t + 1) % M], v[t], l);
}

__device__ __forceinline__ int64_t gather_source(const Segment &seg, int64_t i, int64_t n,
                                                 bool &bad)
{
    if (!seg.perm) return i;
    const int64_t src = seg.p[i];
    if (src < 0 || src >= n) {
        bad = true;
        return -1;
    }
    return src;
}

// A series' first run of element-wise operations with the entanglement on
// load (see launch_segment_entangle32).
template <int M>
__global__ __launch_bounds__(kBlock) void k_segment_entangle32(PtrsI32 c, Segment seg, PtrsW32 y,
                                                               int count, int64_t n, int l,
                                                               uint32_t *err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        int32_t e[M];
        entangle_slots32<M, M>(c, gather_source(seg, i, n, bad), l, e);
        segment_ops_all<int32_t, M>(e, seg, i);
#pragma unroll
        for (int t = 0; t < M; ++t)
            if (t < count) y.p[t][i] = e[t];
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

// A series' last run of element-wise operations with the recovery (see
// launch_segment_extract32).
template <int M, bool ENT>
__global__ __launch_bounds__(kBlock) void k_segment_extract32(PtrsI32 in, PtrsI32 c, Segment seg,
                                                              PtrsW32 out, int64_t n, int l,
                                                              uint32_t *err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t src = gather_source(seg, i, n, bad);
        int32_t a[M - 1], o[M];
        if (ENT) {
            entangle_slots32<M, M - 1>(c, src, l, a);
        } else if (seg.rows > 0) {
#pragma unroll
            for (int t = 0; t < M - 1; ++t) a[t] = src >= 0 ? in.p[0][src * seg.rows + t] : 0;
        } else {
#pragma unroll
            for (int t = 0; t < M - 1; ++t) a[t] = src >= 0 ? in.p[t][src] : 0;
        }
        segment_ops_all<int32_t, M - 1>(a, seg, i);
        recover32<M>(a, o, l);
#pragma unroll
        for (int t = 0; t < M; ++t) out.p[t][i] = o[t];
    }
    if (bad && err) atomicOr(err, NE_FLAG_PERM_INDEX);
}

template <int M>
void segment_entangle32_m(int l, int64_t n, int count, const PtrsI32 &c, const Segment &seg,
                          const PtrsW32 &y, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL(k_segment_entangle32<M>, dim3(grid_for(n)), dim3(kBlock), 0, s, c, seg, y,
                       count, n, l, err);
}

template <int M>
void segment_extract32_m(int l, int64_t n, bool entangle, const PtrsI32 &in, const PtrsI32 &c,
                         const Segment &seg, const PtrsW32 &out, uint32_t *err, hipStream_t s)
{
    if (entangle)
        hipLaunchKernelGGL((k_segment_extract32<M, true>), dim3(grid_for(n)), dim3(kBlock), 0, s,
                           in, c, seg, out, n, l, err);
    else
        hipLaunchKernelGGL((k_segment_extract32<M, false>), dim3(grid_for(n)), dim3(kBlock), 0, s,
                           in, c, seg, out, n, l, err);
}

}  // namespace

void launch_segment_entangle32(int M, int l, int64_t n, int count, const PtrsI32 &c,
                               const Segment &seg, const PtrsW32 &y, uint32_t *err, hipStream_t s)
{
    NE_DISPATCH_M32(M, segment_entangle32_m, l, n, count, c, seg, y, err, s);
}

void launch_segment_extract32(int M, int l, int64_t n, bool entangle, const PtrsI32 &in,
                              const PtrsI32 &c, const Segment &seg, const PtrsW32 &out,
                              uint32_t *err, hipStream_t s)
{
    NE_DISPATCH_M32(M, segment_extract32_m, l, n, entangle, in, c, seg, out, err, s);
}

void launch_extract32(int M, int l, int64_t n, const PtrsI32 &in, const PtrsW32 &out, hipStream_t s)
{
    NE_DISPATCH_M32(M, extract32_m, l, n, in, out, s);
}

void launch_conv32_rows(int32_t op, int count, int64_t n_in, const PtrsI32 &x,
                        const int32_t *operand, int64_t n_operand, int64_t n_out, int32_t *rows,
                        hipStream_t s)
{
    const int kind =
        op == NE_OP_CIRC ? kConvCircular : (op == NE_OP_XCORR ? kConvXcorr : kConvLinear);
    PtrsW32 y{};
    y.p[0] = rows;
    ConvArgs32 a{x, y, operand, n_in, n_operand, n_out, kind, count};
    hipLaunchKernelGGL(k_conv32, dim3((unsigned)((n_out + kTile - 1) / kTile), count),
                       dim3(kBlock), 0, s, a);
}

void launch_op32(int32_t op, int count, int64_t n_in, const PtrsI32 &x, const int32_t *operand,
                 int64_t n_operand, int64_t scalar, const PtrsW32 &y, int64_t n_out,
                 hipStream_t s)
{
    const uint32_t sv = (uint32_t)(uint64_t)scalar;
    switch (op) {
    case NE_OP_SCALE: map32<kMapScale>(count, n_in, x, nullptr, y, sv, s); break;
    case NE_OP_ADD: map32<kMapAdd>(count, n_in, x, operand, y, 0, s); break;
    case NE_OP_SUB: map32<kMapSub>(count, n_in, x, operand, y, 0, s); break;
    case NE_OP_MUL: map32<kMapMul>(count, n_in, x, operand, y, 0, s); break;
    case NE_OP_PERM:
        hipLaunchKernelGGL(k_perm32, dim3(grid_for(n_in, kBlock, 4096), count), dim3(kBlock), 0,
                           s, x, operand, y, n_in, device_flag_word());
        break;
    case NE_OP_INNER:
        hipLaunchKernelGGL(k_zero_first32, dim3(count), dim3(64), 0, s, y);
        hipLaunchKernelGGL(k_inner32, dim3(grid_for(n_in, kBlock * 8, 1024), count), dim3(kBlock),
                           0, s, x, operand, y, n_in);
        break;
    case NE_OP_OUTER:
        hipLaunchKernelGGL(k_outer32, dim3(grid_for(n_out, kBlock, 4096), count), dim3(kBlock), 0,
                           s, x, operand, y, n_in, n_operand);
        break;
    default: {  // NE_OP_CONV, NE_OP_CIRC, NE_OP_XCORR
        const int kind =
            op == NE_OP_CIRC ? kConvCircular : (op == NE_OP_XCORR ? kConvXcorr : kConvLinear);
        ConvArgs32 a{x, y, operand, n_in, n_operand, n_out, kind, 0};
        hipLaunchKernelGGL(k_conv32, dim3((unsigned)((n_out + kTile - 1) / kTile), count),
                           dim3(kBlock), 0, s, a);
        break;
    }
    }
}

}  // namespace ne

using namespace ne;

namespace {

// l and (M - 1) l that the 32-bit extraction accepts: every word's low
// (M - 1) l bits must fit the register.
inline bool bad_l32(int32_t M, int32_t l) { return l < 1 || l > 31 || (M - 1) * l > 32; }

}  // namespace

extern "C" {

ne_status ne_entangle32(int32_t M, int32_t l, int64_t n, const int32_t *const *c,
                        int32_t *const *eps, ne_stream stream)
{
    if (M < 3 || M > NE_MAX_M32 || l < 1 || l > 31 || n < 0 || !c || !eps) return NE_EINVAL;
    if (n == 0) return NE_OK;
    PtrsI32 pc{};
    PtrsW32 pe{};
    for (int m = 0; m < M; ++m) {
        if (!c[m] || !eps[m]) return NE_EINVAL;
        pc.p[m] = c[m];
        pe.p[m] = eps[m];
    }
    NE_DISPATCH_M32(M, entangle32_m, l, n, pc, pe, (hipStream_t)stream);
    return launch_status();
}

ne_status ne_entangle_operand32(int32_t l, int64_t n, const int32_t *g, int32_t *g_ent,
                                ne_stream stream)
{
    if (l < 1 || l > 31 || n < 0) return NE_EINVAL;
    if (n == 0) return NE_OK;
    if (!g || !g_ent) return NE_EINVAL;
    hipLaunchKernelGGL(k_entangle_operand32, dim3(grid_for(n)), dim3(kBlock), 0,
                       (hipStream_t)stream, g, g_ent, n, l);
    return launch_status();
}

ne_status ne_lsb_apply32(int32_t op, int32_t M, int64_t n_in, const int32_t *const *eps,
                         const int32_t *operand, int64_t n_operand, int64_t scalar,
                         int32_t *const *delta, int64_t n_out, uint32_t stream_mask,
                         ne_stream stream)
{
    if (M < 1 || M > NE_MAX_M || !eps || !delta) return NE_EINVAL;
    const ne_status st = check_op_shape(op, n_in, operand, n_operand, n_out);
    if (st != NE_OK) return st;
    if (M < 32) stream_mask &= (1u << M) - 1u;
    PtrsI32 px{};
    PtrsW32 py{};
    int count = 0;
    for (int m = 0; m < M; ++m) {
        if (!((stream_mask >> m) & 1u)) continue;
        if ((!eps[m] && n_in > 0) || (!delta[m] && n_out > 0)) return NE_EINVAL;
        px.p[count] = eps[m];
        py.p[count] = delta[m];
        ++count;
    }
    if (count == 0 || n_out == 0) return NE_OK;
    launch_op32(op, count, n_in, px, operand, n_operand, scalar, py, n_out,
                (hipStream_t)stream);
    return launch_status();
}

ne_status ne_extract_recover32(int32_t M, int32_t l, int64_t n_out, const int32_t *const *delta,
                               int32_t r, int32_t *const *dhat, ne_stream stream)
{
    if (M < 3 || M > NE_MAX_M32 || bad_l32(M, l) || n_out < 0 || !delta || !dhat)
        return NE_EINVAL;
    if (r < -1 || r >= M) return NE_EFAILIDX;
    if (n_out == 0) return NE_OK;
    if (r < 0) r = 0;
    PtrsI32 in{};
    PtrsW32 out{};
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
    NE_DISPATCH_M32(M, extract32_m, l, n_out, in, out, (hipStream_t)stream);
    return launch_status();
}

}  // extern "C"
