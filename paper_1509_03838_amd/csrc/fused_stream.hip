// Fused element-wise kernel variants of one kernel class (-DNE_KCLASS=k):
// scale, add, inner product, permutation, subtraction, element-by-element
// product and outer product for every slot count the class
// has (entangled 3..8, plain 1..8, checksum 3..9).
#include "fused_kernels.h"

#if !defined(NE_KCLASS)
#error "NE_KCLASS selects the kernel class of this translation unit"
#endif

#define NE_CAT2(a, b) a##b
#define NE_NAME(a, b) NE_CAT2(a, b)

namespace ne {

namespace {

constexpr int kLo = NE_KCLASS == 1 ? 1 : 3;
constexpr int kHi = NE_KCLASS == 2 ? 9 : 8;

template <int OP, int NS>
void launch_one(const GroupDev *g, const Item *items, uint32_t nitems, uint32_t *flags,
                hipStream_t s)
{
    constexpr int VX = stream_positions_of(OP, NS) / stream_positions(NS);
    hipLaunchKernelGGL((fk::k_stream_fused<OP, NE_KCLASS, NS, VX>), dim3(nitems), dim3(fk::kBlock),
                       0, s, g, items, nitems, flags);
}

template <int OP, int NS>
constexpr StreamLaunch entry()
{
    if constexpr (NS >= kLo && NS <= kHi)
        return &launch_one<OP, NS>;
    else
        return nullptr;
}

#define NE_ROW(OP)                                                                           \
    {entry<OP, 1>(), entry<OP, 2>(), entry<OP, 3>(), entry<OP, 4>(), entry<OP, 5>(),       \
     entry<OP, 6>(), entry<OP, 7>(), entry<OP, 8>(), entry<OP, 9>()}
// rows: scale, add, inner product, permutation, subtraction, product
// (NE_OP_SCALE .. NE_OP_MUL), then the outer product
const StreamLaunch table[7][kMaxSlots] = {NE_ROW(NE_OP_SCALE), NE_ROW(NE_OP_ADD),
                                          NE_ROW(NE_OP_INNER), NE_ROW(NE_OP_PERM),
                                          NE_ROW(NE_OP_SUB),   NE_ROW(NE_OP_MUL),
                                          NE_ROW(NE_OP_OUTER)};
#undef NE_ROW

}  // namespace

StreamLaunch NE_NAME(stream_kernel_, NE_KCLASS)(int op, int slots)
{
    if (slots < 1 || slots > kMaxSlots) return nullptr;
    if (op == NE_OP_OUTER) return table[6][slots - 1];
    if (op < NE_OP_SCALE || op > NE_OP_MUL) return nullptr;
    return table[op - NE_OP_SCALE][slots - 1];
}

}  // namespace ne
