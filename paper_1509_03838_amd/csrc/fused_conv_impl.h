// Instantiation of the convolution kernel for one slot capacity NS over
// every digit-count pair (LA, LB); included once per capacity so that the
// instantiations compile in parallel translation units.
#pragma once

#include "fused_kernels.h"

namespace ne {

namespace {
template <int LA, int LB, int NS>
void conv_launch_one(const GroupDev *g, const Item *items, uint32_t nitems, uint32_t *flags,
                     size_t lds, hipStream_t s)
{
    const uint32_t grid = ((nitems + 7u) >> 3) << 3;
    hipLaunchKernelGGL((fk::k_conv_fused<LA, LB, NS>), dim3(grid), dim3(fk::kBlock), lds, s, g,
                       items, nitems, flags);
}

template <int LA, int LB, int NS>
hipError_t conv_lds_one(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&fk::k_conv_fused<LA, LB, NS>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

using LaunchFn = void (*)(const GroupDev *, const Item *, uint32_t, uint32_t *, size_t,
                          hipStream_t);
using LdsFn = hipError_t (*)(size_t);

#define NE_ROW(F, LA, NS) {F<LA, 1, NS>, F<LA, 2, NS>, F<LA, 3, NS>, F<LA, 4, NS>}
#define NE_TABLE(F, NS)                                                                    \
    {NE_ROW(F, 1, NS), NE_ROW(F, 2, NS), NE_ROW(F, 3, NS), NE_ROW(F, 4, NS),               \
     NE_ROW(F, 5, NS), NE_ROW(F, 6, NS), NE_ROW(F, 7, NS), NE_ROW(F, 8, NS)}
}  // namespace

template <int NS>
hipError_t conv_prepare_ns(int la, int lb, size_t lds)
{
    static const LdsFn table[kLimbsA][kLimbsB] = NE_TABLE(conv_lds_one, NS);
    return table[la - 1][lb - 1](lds);
}

template <int NS>
void conv_launch_ns(int la, int lb, const GroupDev *g, const Item *items, uint32_t nitems,
                    uint32_t *flags, size_t lds, hipStream_t s)
{
    static const LaunchFn table[kLimbsA][kLimbsB] = NE_TABLE(conv_launch_one, NS);
    table[la - 1][lb - 1](g, items, nitems, flags, lds, s);
}

}  // namespace ne
