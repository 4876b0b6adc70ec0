// Measured ceilings of the fused kernels: the memory-bandwidth reference
// (ne_stream_widen), a copy with their read:write mix and access widths and
// none of the method's arithmetic, and the i8 matrix-core rate
// (ne_mfma_i8_peak), back-to-back products with nothing else to wait for.
#include "ne_internal.h"

namespace {

constexpr int kWidenBlock = 256;
constexpr int kWidenTile = 4 * kWidenBlock;  // elements per block step: 4 KiB in, 8 KiB out
constexpr int kWidenTiles = 2;               // steps per block (their loads issued together)

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef long v2l __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v2i gcv2i_t;
typedef __attribute__((address_space(1))) v2l gv2l_t;

// out[i] = (int64) in[i]. A block step covers kWidenTile elements in two
// halves; in each half thread t reads elements 2t, 2t + 1 (one 8-byte load:
// a wave's load covers 512 contiguous bytes) and writes them as one 16-byte
// non-temporal store (a wave's store covers 1 KiB). Every load of the
// block's kWidenTiles steps is issued before the first store. The last,
// partial step goes element by element.
__global__ __launch_bounds__(kWidenBlock) void k_widen(const int32_t *__restrict__ in,
                                                       int64_t *__restrict__ out, int64_t n)
{
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kWidenTile * kWidenTiles;
    if (base + kWidenTile * kWidenTiles <= n) {
        v2i v[kWidenTiles][2];
#pragma unroll
        for (int s = 0; s < kWidenTiles; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                v[s][h] = *(gcv2i_t *)(in + base + s * kWidenTile + h * (kWidenTile / 2) + 2 * t);
#pragma unroll
        for (int s = 0; s < kWidenTiles; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const v2l w = {(long)v[s][h].x, (long)v[s][h].y};
                __builtin_nontemporal_store(
                    w, (gv2l_t *)(out + base + s * kWidenTile + h * (kWidenTile / 2) + 2 * t));
            }
        return;
    }
    for (int64_t i = base + t; i < n && i < base + kWidenTile * kWidenTiles; i += kWidenBlock)
        out[i] = in[i];
}

// Every wave issues `iters` rounds of kChains independent
// v_mfma_i32_16x16x64_i8 on register operands; the accumulators are folded
// into one word per wave at the end, so no product can be dropped. With
// `varied` false the operands stay the same for every product; with it true
// each product of a round takes another of kChains A and 2 B operands filled
// with pseudo-random bytes (a different pair every product, as digit planes
// of data are), which is what the matrix cores' power draw, and so their
// sustained rate, depends on.
constexpr int kChains = 8;
__device__ __forceinline__ int hash_word(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return (int)x;
}
__global__ __launch_bounds__(256) void k_mfma_i8_peak(int64_t iters, int32_t varied,
                                                      int32_t *__restrict__ sink)
{
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    v4i a[kChains], b[2];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            a[c][e] = varied ? hash_word(gid * 64u + c * 4u + e) : (int)(gid + c * 0x01010101u + e);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            b[c][e] = varied ? hash_word(gid * 64u + 40u + c * 4u + e) : (int)(gid * 7u + 5u + e);
    v4i acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = v4i{c, 0, 0, 0};
    if (varied) {
        // rounds in sets of 8 (iters is a multiple of 8): round r pairs chain c
        // with A operand (c + r) mod 8, so consecutive products differ
        for (int64_t i = 0; i < iters; i += 8) {
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[(c + r) & 7], b[(c + r) & 1],
                                                                  acc[c], 0, 0, 0);
        }
    } else {
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], b[0], acc[c], 0, 0, 0);
        }
    }
    int32_t t = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) t += acc[c].x + acc[c].y + acc[c].z + acc[c].w;
    sink[blockIdx.x * 4 + (threadIdx.x >> 6)] = t;
}

}  // namespace

extern "C" ne_status ne_mfma_i8_peak(int32_t blocks, int64_t iters, int32_t varied, int32_t *sink,
                                     double *ops, ne_stream stream)
{
    if (blocks < 1 || iters < 1 || !sink || (varied && iters % 8)) return NE_EINVAL;
    if (ops) *ops = 2.0 * 16 * 16 * 64 * (double)kChains * (double)iters * 4.0 * blocks;
    hipLaunchKernelGGL(k_mfma_i8_peak, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       iters, varied, sink);
    return ne::launch_status();
}

extern "C" ne_status ne_stream_widen(const int32_t *in, int64_t n, int64_t *out,
                                     ne_stream stream)
{
    if (n < 0) return NE_EINVAL;
    if (n == 0) return NE_OK;
    if (!in || !out || ((uintptr_t)in % 16) || ((uintptr_t)out % 16)) return NE_EINVAL;
    if ((uintptr_t)out < (uintptr_t)(in + n) && (uintptr_t)in < (uintptr_t)(out + n))
        return NE_EINVAL;
    const int64_t per = (int64_t)kWidenTile * kWidenTiles;
    const int64_t grid = (n + per - 1) / per;
    if (grid > 0x7fffffff) return NE_EUNSUP;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)grid), dim3(kWidenBlock), 0, (hipStream_t)stream,
                       in, out, n);
    return ne::launch_status();
}
