// Device-side descriptors of the batched executor (private to libne).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ne {

constexpr int kFusedMaxM = 8;       // data streams per group in the fused kernels
constexpr int kMaxSlots = kFusedMaxM + 1;  // + the checksum stream
constexpr int kConvTile = 1024;     // output positions per block step (4 waves x 256)
constexpr int kLimbsA = 8;          // largest limb count of a data word
constexpr int kLimbsB = 4;          // largest limb count of an operand value
constexpr int kStreamV0 = 4;        // element-wise kernel: positions per lane, <= 4 slots
constexpr int kStreamV1 = 2;        // element-wise kernel: positions per lane, <= 9 slots

// Execution modes of a plan.
enum Mode : int32_t {
    kEntangled = 0,  // the method: entangle, op per stream, extract
    kPlain = 1,      // failure-intolerant op on the raw streams, narrow limbs
    kPlainSame = 2,  // failure-intolerant op on the same datapath as kEntangled
    kChecksum = 3    // checksum method: M data streams + their sum
};

// Error bits reported through the plan's flag word.
enum Flag : uint32_t {
    kFlagInputRange = 1u,   // an input or operand value outside the declared bits
    kFlagLimbs = 2u,        // a word did not fit the chosen limb count
    kFlagMismatch = 4u      // the redundant stream disagreed with the recovered outputs
};

struct GroupDev {
    int32_t op;       // NE_OP_*
    int32_t M;        // data streams
    int32_t mode;     // Mode
    int32_t r;        // stream left out of recovery (the lost one, else 0)
    int32_t lost;     // 1 if stream r was lost (its operation is not run)
    int32_t l;        // shift (entangled mode)
    int32_t la, lb;   // limbs of data words / operand values (conv)
    int32_t nslots;   // streams whose operation runs: M, or M + 1 (checksum)
    int32_t nch;      // 64-wide chunks of the inner dimension (conv)
    int32_t kp;       // window lead: 64 * nch - 16 (conv)
    int32_t wlen;     // staged window length: kConvTile + kp (conv)
    int32_t in_lo, in_hi;  // declared input range [in_lo, in_hi]
    int32_t steps;    // conv tile steps (or streaming positions / 256) per block
    int32_t ring;     // bytes per LDS digit-plane ring (= wlen) (conv)
    int32_t acc16;    // 1: every acc_s + 256 acc_{s+1} fits in int32 (conv)
    int32_t dma;      // 1: next-step inputs are prefetched into LDS (conv)
    int64_t n, K, n_out;
    int64_t scalar;
    const int32_t *c[kFusedMaxM];
    const int32_t *operand;
    int64_t *out[kFusedMaxM];
    uint64_t *acc;    // inner product: kMaxSlots accumulators
};

struct Item {
    uint32_t g;       // group index
    uint32_t strip;   // strip index within the group
};

// Launchers of the fused kernels (fused_conv*.hip, fused.hip).
template <int NS>
hipError_t conv_prepare_ns(int la, int lb, size_t lds);
template <int NS>
void conv_launch_ns(int la, int lb, const GroupDev *g, const Item *items, uint32_t nitems,
                    uint32_t *flags, size_t lds, hipStream_t s);
hipError_t fused_conv_prepare(int cls, int la, int lb, size_t lds);
void fused_conv_launch(int cls, int la, int lb, const GroupDev *g, const Item *items,
                       uint32_t nitems, uint32_t *flags, size_t lds, hipStream_t s);
void fused_stream_launch(int cls, const GroupDev *g, const Item *items, uint32_t nitems,
                         uint32_t *flags, hipStream_t s);
void fused_inner_finalize(const GroupDev *g, const uint32_t *gidx, uint32_t count,
                          uint32_t *flags, hipStream_t s);

}  // namespace ne
