// Fused convolution kernel variants of one kernel class and slot count,
// selected at compile time (-DNE_KCLASS=k -DNE_SLOTS=n): every digit-count
// pair (LA, LB) and shape that some group of that class and slot count can
// need.
#include "conv_variants.h"
#include "fused_kernels.h"

#if !defined(NE_KCLASS) || !defined(NE_SLOTS)
#error "NE_KCLASS and NE_SLOTS select the variants of this translation unit"
#endif

#define NE_CAT3(a, b, c) a##b##_##c
#define NE_NAME(a, b, c) NE_CAT3(a, b, c)

namespace ne {

namespace {

// Shape V of a variant: 0 plain digits, 1 sparse top tap digit, 2 data words
// split into two fields of LA / 2 digits.
constexpr int sp_of(int v) { return v == 1 ? 1 : 0; }
constexpr int fs_of(int la, int v) { return v == 2 ? la / 2 : 0; }

template <int LA, int LB, int L, int SP>
void launch_one(const GroupDev *g, const Item *items, uint32_t nitems, uint32_t *flags,
                size_t lds, hipStream_t s)
{
    const uint32_t grid = ((nitems + 7u) >> 3) << 3;
    hipLaunchKernelGGL((fk::k_conv_fused<LA, LB, NE_SLOTS, NE_KCLASS, conv_layout_waves(L),
                                         sp_of(SP), conv_layout_copies(L), fs_of(LA, SP)>),
                       dim3(grid),
                       dim3(fk::kBlock), lds, s, g, items, nitems, flags);
}

template <int LA, int LB, int L, int SP>
const void *kernel_of()
{
    return reinterpret_cast<const void *>(
        &fk::k_conv_fused<LA, LB, NE_SLOTS, NE_KCLASS, conv_layout_waves(L), sp_of(SP),
                          conv_layout_copies(L), fs_of(LA, SP)>);
}

template <int LA, int LB, int L, int SP>
hipError_t prepare_one(size_t lds)
{
    return hipFuncSetAttribute(kernel_of<LA, LB, L, SP>(),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int LA, int LB, int L, int SP>
hipError_t attributes_one(hipFuncAttributes *a)
{
    return hipFuncGetAttributes(a, kernel_of<LA, LB, L, SP>());
}

using LaunchFn = void (*)(const GroupDev *, const Item *, uint32_t, uint32_t *, size_t,
                          hipStream_t);
using PrepareFn = hipError_t (*)(size_t);
using AttributesFn = hipError_t (*)(hipFuncAttributes *);

template <int LA, int LB, int SP>
constexpr bool needed()
{
    if constexpr ((SP == 1 && LB < 2) || (SP == 2 && LA % 2 != 0))
        return false;
    else
        return conv_variant_needed(NE_KCLASS, NE_SLOTS, LA, LB, SP);
}

template <int LA, int LB, int L, int SP>
constexpr LaunchFn launcher()
{
    if constexpr (needed<LA, LB, SP>())
        return &launch_one<LA, LB, L, SP>;
    else
        return nullptr;
}

template <int LA, int LB, int L, int SP>
constexpr PrepareFn preparer()
{
    if constexpr (needed<LA, LB, SP>())
        return &prepare_one<LA, LB, L, SP>;
    else
        return nullptr;
}

template <int LA, int LB, int L, int SP>
constexpr AttributesFn attributer()
{
    if constexpr (needed<LA, LB, SP>())
        return &attributes_one<LA, LB, L, SP>;
    else
        return nullptr;
}

template <int LA, int LB>
constexpr ConvKernel entry()
{
    return ConvKernel{
        {{launcher<LA, LB, 0, 0>(), launcher<LA, LB, 1, 0>(), launcher<LA, LB, 2, 0>()},
         {launcher<LA, LB, 0, 1>(), launcher<LA, LB, 1, 1>(), launcher<LA, LB, 2, 1>()},
         {launcher<LA, LB, 0, 2>(), launcher<LA, LB, 1, 2>(), launcher<LA, LB, 2, 2>()}},
        {{preparer<LA, LB, 0, 0>(), preparer<LA, LB, 1, 0>(), preparer<LA, LB, 2, 0>()},
         {preparer<LA, LB, 0, 1>(), preparer<LA, LB, 1, 1>(), preparer<LA, LB, 2, 1>()},
         {preparer<LA, LB, 0, 2>(), preparer<LA, LB, 1, 2>(), preparer<LA, LB, 2, 2>()}},
        {{attributer<LA, LB, 0, 0>(), attributer<LA, LB, 1, 0>(), attributer<LA, LB, 2, 0>()},
         {attributer<LA, LB, 0, 1>(), attributer<LA, LB, 1, 1>(), attributer<LA, LB, 2, 1>()},
         {attributer<LA, LB, 0, 2>(), attributer<LA, LB, 1, 2>(), attributer<LA, LB, 2, 2>()}}};
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
    return (k->launch[0][0] || k->launch[1][0] || k->launch[2][0]) ? k : nullptr;
}

}  // namespace ne
