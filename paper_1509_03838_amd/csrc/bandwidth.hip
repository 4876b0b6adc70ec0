// The memory-bandwidth reference of the fused kernels (ne_stream_widen): a
// copy with their read:write mix and access widths and none of the method's
// arithmetic, so that its rate is the practical HBM ceiling a fused
// convolution can be held to.
#include "ne_internal.h"

namespace {

constexpr int kWidenBlock = 256;
constexpr int kWidenTile = 4 * kWidenBlock;  // elements per block step: 4 KiB in, 8 KiB out
constexpr int kWidenTiles = 2;               // steps per block (their loads issued together)

typedef int v2i __attribute__((ext_vector_type(2)));
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

}  // namespace

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
