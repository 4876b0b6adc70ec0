// Fused convolution kernel variants of one kernel class and slot count,
// selected at compile time (-DNE_KCLASS=k -DNE_SLOTS=n): every digit-count
// pair (LA, LB) that some group of that class and slot count can need.
#include "conv_variants.h"
#include "fused_kernels.h"

#if !defined(NE_KCLASS) || !defined(NE_SLOTS)
#error "NE_KCLASS and NE_SLOTS select the variants of this translation unit"
#endif

#define NE_CAT3(a, b, c) a##b##_##c
#define NE_NAME(a, b, c) NE_CAT3(a, b, c)

namespace ne {

namespace {

template <int LA, int LB, int GW>
void launch_one(const GroupDev *g, const Item *items, uint32_t nitems, uint32_t *flags,
                size_t lds, hipStream_t s)
{
    const uint32_t grid = ((nitems + 7u) >> 3) << 3;
    hipLaunchKernelGGL((fk::k_conv_fused<LA, LB, NE_SLOTS, NE_KCLASS, GW>), dim3(grid),
                       dim3(fk::kBlock), lds, s, g, items, nitems, flags);
}

template <int LA, int LB, int GW>
hipError_t prepare_one(size_t lds)
{
    return hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fk::k_conv_fused<LA, LB, NE_SLOTS, NE_KCLASS, GW>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int LA, int LB>
constexpr ConvKernel entry()
{
    if constexpr (conv_variant_needed(NE_KCLASS, NE_SLOTS, LA, LB))
        return ConvKernel{{&launch_one<LA, LB, 4>, &launch_one<LA, LB, 1>},
                          {&prepare_one<LA, LB, 4>, &prepare_one<LA, LB, 1>}};
    else
        return ConvKernel{{nullptr, nullptr}, {nullptr, nullptr}};
}

#define NE_ROW(LA) {entry<LA, 1>(), entry<LA, 2>(), entry<LA, 3>(), entry<LA, 4>()}
const ConvKernel table[kLimbsA][kLimbsB] = {NE_ROW(1), NE_ROW(2), NE_ROW(3), NE_ROW(4),
                                            NE_ROW(5), NE_ROW(6), NE_ROW(7), NE_ROW(8)};
#undef NE_ROW

}  // namespace

const ConvKernel *NE_NAME(conv_kernel_, NE_KCLASS, NE_SLOTS)(int la, int lb)
{
    if (la < 1 || la > kLimbsA || lb < 1 || lb > kLimbsB) return nullptr;
    const ConvKernel *k = &table[la - 1][lb - 1];
    return k->launch[0] ? k : nullptr;
}

}  // namespace ne
