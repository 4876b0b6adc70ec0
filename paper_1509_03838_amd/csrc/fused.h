// Device-side descriptors of the batched executor (private to libne).
#pragma once

#include <stdint.h>

namespace ne {

constexpr int kFusedMaxM = 8;       // data streams per group in the fused kernels
constexpr int kMaxSlots = kFusedMaxM + 1;  // + the checksum stream
constexpr int kConvTile = 1024;     // output positions per block step (4 waves x 256)
constexpr int kLimbsA = 8;          // largest limb count of a data word
constexpr int kLimbsB = 4;          // largest limb count of an operand value

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
    int32_t pad_;
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

}  // namespace ne
