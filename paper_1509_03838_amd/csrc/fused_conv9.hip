// Convolution kernels for groups of up to 9 slots (M <= 8, plus the checksum
// stream).
#include "fused_conv_impl.h"

namespace ne {
template hipError_t conv_prepare_ns<kMaxSlots>(int, int, size_t);
template void conv_launch_ns<kMaxSlots>(int, int, const GroupDev *, const Item *, uint32_t,
                                        uint32_t *, size_t, hipStream_t);
}  // namespace ne
