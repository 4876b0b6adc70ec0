// Launchers of the fused element-wise kernels and dispatch of the fused
// convolution kernels by slot capacity.
#include "fused_kernels.h"

namespace ne {

hipError_t fused_conv_prepare(int cls, int la, int lb, size_t lds)
{
    return cls == 0 ? conv_prepare_ns<4>(la, lb, lds) : conv_prepare_ns<kMaxSlots>(la, lb, lds);
}

void fused_conv_launch(int cls, int la, int lb, const GroupDev *g, const Item *items,
                       uint32_t nitems, uint32_t *flags, size_t lds, hipStream_t s)
{
    if (cls == 0)
        conv_launch_ns<4>(la, lb, g, items, nitems, flags, lds, s);
    else
        conv_launch_ns<kMaxSlots>(la, lb, g, items, nitems, flags, lds, s);
}

void fused_stream_launch(int cls, const GroupDev *g, const Item *items, uint32_t nitems,
                         uint32_t *flags, hipStream_t s)
{
    if (cls == 0)
        hipLaunchKernelGGL((fk::k_stream_fused<4, kStreamV0>), dim3(nitems), dim3(fk::kBlock), 0, s,
                           g, items, nitems, flags);
    else
        hipLaunchKernelGGL((fk::k_stream_fused<kMaxSlots, kStreamV1>), dim3(nitems),
                           dim3(fk::kBlock), 0, s, g, items, nitems, flags);
}

void fused_inner_finalize(const GroupDev *g, const uint32_t *gidx, uint32_t count,
                          uint32_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(fk::k_inner_finalize<kMaxSlots>, dim3((count + 63) / 64), dim3(64), 0, s,
                       g, gidx, count, flags);
}

}  // namespace ne
