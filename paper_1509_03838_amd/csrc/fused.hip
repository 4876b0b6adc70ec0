// Launchers of the fused element-wise kernels and lookup of the fused
// convolution kernel variants.
#include "fused_kernels.h"

namespace ne {

// Variants built by fused_conv.hip: entangled groups of 3..8 streams, plain
// groups of 1..8, checksum groups of 2..8 data streams (3..9 slots).
const ConvKernel *conv_kernel_0_3(int la, int lb);
const ConvKernel *conv_kernel_0_4(int la, int lb);
const ConvKernel *conv_kernel_0_5(int la, int lb);
const ConvKernel *conv_kernel_0_6(int la, int lb);
const ConvKernel *conv_kernel_0_7(int la, int lb);
const ConvKernel *conv_kernel_0_8(int la, int lb);
const ConvKernel *conv_kernel_1_1(int la, int lb);
const ConvKernel *conv_kernel_1_2(int la, int lb);
const ConvKernel *conv_kernel_1_3(int la, int lb);
const ConvKernel *conv_kernel_1_4(int la, int lb);
const ConvKernel *conv_kernel_1_5(int la, int lb);
const ConvKernel *conv_kernel_1_6(int la, int lb);
const ConvKernel *conv_kernel_1_7(int la, int lb);
const ConvKernel *conv_kernel_1_8(int la, int lb);
const ConvKernel *conv_kernel_2_3(int la, int lb);
const ConvKernel *conv_kernel_2_4(int la, int lb);
const ConvKernel *conv_kernel_2_5(int la, int lb);
const ConvKernel *conv_kernel_2_6(int la, int lb);
const ConvKernel *conv_kernel_2_7(int la, int lb);
const ConvKernel *conv_kernel_2_8(int la, int lb);
const ConvKernel *conv_kernel_2_9(int la, int lb);

const ConvKernel *conv_kernel(int kclass, int slots, int la, int lb)
{
    switch (kclass * 16 + slots) {
    case 3: return conv_kernel_0_3(la, lb);
    case 4: return conv_kernel_0_4(la, lb);
    case 5: return conv_kernel_0_5(la, lb);
    case 6: return conv_kernel_0_6(la, lb);
    case 7: return conv_kernel_0_7(la, lb);
    case 8: return conv_kernel_0_8(la, lb);
    case 17: return conv_kernel_1_1(la, lb);
    case 18: return conv_kernel_1_2(la, lb);
    case 19: return conv_kernel_1_3(la, lb);
    case 20: return conv_kernel_1_4(la, lb);
    case 21: return conv_kernel_1_5(la, lb);
    case 22: return conv_kernel_1_6(la, lb);
    case 23: return conv_kernel_1_7(la, lb);
    case 24: return conv_kernel_1_8(la, lb);
    case 35: return conv_kernel_2_3(la, lb);
    case 36: return conv_kernel_2_4(la, lb);
    case 37: return conv_kernel_2_5(la, lb);
    case 38: return conv_kernel_2_6(la, lb);
    case 39: return conv_kernel_2_7(la, lb);
    case 40: return conv_kernel_2_8(la, lb);
    case 41: return conv_kernel_2_9(la, lb);
    default: return nullptr;
    }
}

// Element-wise variants built by fused_stream.hip (one translation unit per
// kernel class).
StreamLaunch stream_kernel_0(int op, int slots);
StreamLaunch stream_kernel_1(int op, int slots);
StreamLaunch stream_kernel_2(int op, int slots);

StreamLaunch stream_kernel(int op, int kclass, int slots)
{
    switch (kclass) {
    case 0: return stream_kernel_0(op, slots);
    case 1: return stream_kernel_1(op, slots);
    case 2: return stream_kernel_2(op, slots);
    default: return nullptr;
    }
}

// Single-launch kernels built by fused_single.hip (one translation unit per
// kernel class).
const SingleKernel *single_kernel_0();
const SingleKernel *single_kernel_1();
const SingleKernel *single_kernel_2();

const SingleKernel *single_kernel(int kclass)
{
    switch (kclass) {
    case 0: return single_kernel_0();
    case 1: return single_kernel_1();
    case 2: return single_kernel_2();
    default: return nullptr;
    }
}

void fused_interleave_launch(int cls, const GroupDev *g, const Item *items, uint32_t nitems,
                             hipStream_t s)
{
    if (cls == 0)
        hipLaunchKernelGGL((fk::k_interleave<4>), dim3(nitems), dim3(fk::kBlock), 0, s, g, items,
                           nitems);
    else
        hipLaunchKernelGGL((fk::k_interleave<8>), dim3(nitems), dim3(fk::kBlock), 0, s, g, items,
                           nitems);
}

void fused_inner_finalize(const GroupDev *g, const uint32_t *gidx, uint32_t count,
                          uint32_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(fk::k_inner_finalize<kMaxSlots>, dim3((count + 63) / 64), dim3(64), 0, s,
                       g, gidx, count, flags);
}

}  // namespace ne
