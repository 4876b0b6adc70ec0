// Full linear convolution y[t] = sum_{j<K} g[j] x[t-j] on the vector ALUs,
// one stream per blockIdx.y, for int64 words (entangled or widened plain
// streams, modulo 2^64) and for raw int32 streams (exact int64 results).
// The same kernels run the circular convolution (the window read modulo
// n, n outputs) and the full cross-correlation (the taps read reversed:
// sum_j g[j] x[t+j-(K-1)] = sum_j g[K-1-j] x[t-j]).
//
// A block owns kTile consecutive outputs. For each chunk of up to kKC taps
// it stages the input window the chunk touches, zero-padded outside
// [0, n), in LDS together with the taps, then every lane accumulates kQ
// outputs spaced kBlock apart, so that consecutive lanes read consecutive
// LDS words (no bank conflicts) and the tap is a broadcast.
//
// In row form (rows > 0) stream t's output i goes to y.p[0][i * rows + t]:
// the rows a permutation gather reads next. The blocks of the streams write
// disjoint words of the same rows (a block that looped over the streams
// measured 2% slower).
//
// int64 x int32 products modulo 2^64 without a 64x64 multiply: the window
// word x is staged as x = xh 2^32 + xs with xs its low half read as a
// signed int32 (xh then carries xs's borrow: xh = (x >> 32) + [xs < 0],
// modulo 2^32), so that
//     x g = xs g + 2^32 (xh g mod 2^32)          (mod 2^64)
// with xs g an exact signed 32x32->64 product. Each tap costs one signed
// 32x32->64 multiply-add into a 64-bit accumulator and one 32-bit
// multiply-add into a second accumulator that only needs to be right
// modulo 2^32; the two are combined once per output. (With an unsigned low
// half the product needs a correction for negative taps, two more vector
// operations per tap and output.)
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kBlock = 256;
constexpr int kQ = 4;
constexpr int kTile = kBlock * kQ;
constexpr int kKC = 1024;

struct ConvArgsI64 {
    PtrsCI64 x;
    PtrsI64 y;
    const int32_t *g;
    int64_t n, K, n_out;
    int32_t kind;  // ConvKind
    int32_t rows;  // 0: stream blockIdx.y's outputs to plane y.p[blockIdx.y]; > 0: to rows
};

struct ConvArgsI32 {
    PtrsI32 x;
    PtrsI64 y;
    const int32_t *g;
    int64_t n, K, n_out;
    int32_t kind, pad_;
};

// Input index of window position idx: zero outside [0, n) (linear), or
// wrapped modulo n (circular, n > 0); -1 marks a zero.
__device__ __forceinline__ int64_t window_index(int64_t idx, int64_t n, int kind)
{
    if (kind == kConvCircular) {
        int64_t r = idx % n;
        return r < 0 ? r + n : r;
    }
    return (idx >= 0 && idx < n) ? idx : -1;
}

__device__ __forceinline__ int32_t tap(const int32_t *g, int64_t j, int64_t K, int kind)
{
    return g[kind == kConvXcorr ? K - 1 - j : j];
}

// One stream's tile of kTile outputs (t0 onwards) into out[t * stride].
__device__ __forceinline__ void conv_i64_tile(const ConvArgsI64 &a, const int64_t *x, int64_t *out,
                                              int64_t stride, int32_t *sxl, uint32_t *sxh,
                                              int32_t *sg)
{
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    uint64_t lo[kQ];
    uint32_t hi[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        lo[q] = 0;
        hi[q] = 0;
    }
    for (int64_t j0 = 0; j0 < a.K; j0 += kKC) {
        const int kc = (int)((a.K - j0) < kKC ? (a.K - j0) : kKC);
        const int64_t wbase = t0 - j0 - (kc - 1);
        const int wlen = kTile + kc - 1;
        __syncthreads();
        for (int w = tid; w < wlen; w += kBlock) {
            const int64_t idx = window_index(wbase + w, a.n, a.kind);
            const uint64_t v = idx >= 0 ? (uint64_t)x[idx] : 0;
            const uint32_t l32 = (uint32_t)v;
            sxl[w] = (int32_t)l32;
            sxh[w] = (uint32_t)(v >> 32) + (l32 >> 31);
        }
        for (int j = tid; j < kc; j += kBlock) sg[j] = tap(a.g, j0 + j, a.K, a.kind);
        __syncthreads();
        // four taps per pass: their window words are read from LDS together
        // (8% faster than one tap per pass)
#pragma unroll 4
        for (int j = 0; j < kc; ++j) {
            const int32_t gj = sg[j];
            const uint32_t gu = (uint32_t)gj;
            const int wb = tid + kc - 1 - j;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int32_t xs = sxl[wb + q * kBlock];
                const uint32_t xh = sxh[wb + q * kBlock];
                lo[q] += (uint64_t)((int64_t)xs * (int64_t)gj);
                hi[q] += xh * gu;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int64_t t = t0 + q * kBlock + tid;
        if (t < a.n_out) out[t * stride] = (int64_t)(lo[q] + ((uint64_t)hi[q] << 32));
    }
}

__global__ __launch_bounds__(kBlock) void k_conv_i64(ConvArgsI64 a)
{
    __shared__ int32_t sxl[kTile + kKC];
    __shared__ uint32_t sxh[kTile + kKC];
    __shared__ int32_t sg[kKC];
    if (a.rows == 0)
        conv_i64_tile(a, a.x.p[blockIdx.y], a.y.p[blockIdx.y], 1, sxl, sxh, sg);
    else
        conv_i64_tile(a, a.x.p[blockIdx.y], a.y.p[0] + blockIdx.y, a.rows, sxl, sxh, sg);
}

__global__ __launch_bounds__(kBlock) void k_conv_i32(ConvArgsI32 a)
{
    __shared__ int32_t sx[kTile + kKC];
    __shared__ int32_t sg[kKC];
    const int tid = threadIdx.x;
    const int32_t *x = a.x.p[blockIdx.y];
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    int64_t acc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = 0;
    for (int64_t j0 = 0; j0 < a.K; j0 += kKC) {
        const int kc = (int)((a.K - j0) < kKC ? (a.K - j0) : kKC);
        const int64_t wbase = t0 - j0 - (kc - 1);
        const int wlen = kTile + kc - 1;
        __syncthreads();
        for (int w = tid; w < wlen; w += kBlock) {
            const int64_t idx = window_index(wbase + w, a.n, a.kind);
            sx[w] = idx >= 0 ? x[idx] : 0;
        }
        for (int j = tid; j < kc; j += kBlock) sg[j] = tap(a.g, j0 + j, a.K, a.kind);
        __syncthreads();
        for (int j = 0; j < kc; ++j) {
            const int64_t gj = sg[j];
            const int wb = tid + kc - 1 - j;
#pragma unroll
            for (int q = 0; q < kQ; ++q) acc[q] += (int64_t)sx[wb + q * kBlock] * gj;
        }
    }
    int64_t *y = a.y.p[blockIdx.y];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int64_t t = t0 + q * kBlock + tid;
        if (t < a.n_out) y[t] = acc[q];
    }
}

}  // namespace

void launch_conv_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                     const PtrsI64 &y, hipStream_t s, int kind)
{
    ConvArgsI64 a{x, y, g, n, K, kind == kConvCircular ? n : n + K - 1, kind, 0};
    const int64_t tiles = (a.n_out + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_conv_i64, dim3((unsigned)tiles, count), dim3(kBlock), 0, s, a);
}

void launch_conv_i64_rows(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                          int64_t *rows, hipStream_t s, int kind)
{
    PtrsI64 y{};
    y.p[0] = rows;
    ConvArgsI64 a{x, y, g, n, K, kind == kConvCircular ? n : n + K - 1, kind, count};
    const int64_t tiles = (a.n_out + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_conv_i64, dim3((unsigned)tiles, count), dim3(kBlock), 0, s, a);
}

void launch_conv_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, int64_t K,
                     const PtrsI64 &y, hipStream_t s, int kind)
{
    ConvArgsI32 a{x, y, g, n, K, kind == kConvCircular ? n : n + K - 1, kind, 0};
    const int64_t tiles = (a.n_out + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_conv_i32, dim3((unsigned)tiles, count), dim3(kBlock), 0, s, a);
}

}  // namespace ne
