// Convolution kernels for groups of up to 4 slots (M <= 4, or M <= 3 with a
// checksum stream).
#include "fused_conv_impl.h"

namespace ne {
template hipError_t conv_prepare_ns<4>(int, int, size_t);
template void conv_launch_ns<4>(int, int, const GroupDev *, const Item *, uint32_t, uint32_t *,
                                size_t, hipStream_t);
}  // namespace ne
