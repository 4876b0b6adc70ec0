// Device-side descriptors of the batched executor (private to libne).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ne.h"

namespace ne {

constexpr int kFusedMaxM = 8;       // data streams per group in the fused kernels
constexpr int kMaxSlots = kFusedMaxM + 1;  // + the checksum stream
constexpr int kConvTile = 1024;     // output positions per block step (4 waves x 256)
constexpr int kLimbsA = 8;          // largest limb count of a data word
constexpr int kLimbsB = 4;          // largest limb count of an operand value
constexpr int kStreamV0 = 4;        // element-wise kernel: positions per lane, <= 4 slots
constexpr int kStreamV1 = 2;        // element-wise kernel: positions per lane, <= 9 slots
constexpr int kInterleaveStep = 1024;  // permutation layout pass: positions per block step

// Element-wise kernel: positions per lane per step for a slot count.
__host__ __device__ constexpr int stream_positions(int slots)
{
    return slots <= 4 ? kStreamV0 : kStreamV1;
}

// Execution modes of a plan.
enum Mode : int32_t {
    kEntangled = 0,  // the method: entangle, op per stream, extract
    kPlain = 1,      // failure-intolerant op on the raw streams, narrow limbs
    kPlainSame = 2,  // failure-intolerant op on the same datapath as kEntangled
    kChecksum = 3,   // checksum method: M data streams + their sum
    kChecksumSame = 4  // the checksum method on the same datapath as kEntangled
};

// Error bits reported through the plan's flag word.
enum Flag : uint32_t {
    kFlagInputRange = 1u,   // an input or operand value outside the declared bits
    kFlagLimbs = 2u,        // reserved: digit counts follow the declared (checked) range
    kFlagMismatch = 4u,     // the redundant stream disagreed with the recovered outputs
    kFlagPermIndex = 8u,    // a permutation index outside [0, n)
    kFlagStall = 16u        // single launch: a wait for another work item exceeded its bound
};

struct GroupDev {
    int32_t op;       // NE_OP_*
    int32_t M;        // data streams
    int32_t mode;     // Mode
    int32_t r;        // stream left out of recovery (the lost one, else 0)
    int32_t lost;     // 1 if stream r was lost (its operation is not run)
    int32_t l;        // shift (entangled mode; split words: the field boundary too)
    int32_t la, lb;   // limbs of data words / operand values (conv)
    int32_t nslots;   // streams whose operation runs: M, or M + 1 (checksum)
    int32_t nch;      // 64-wide chunks of the inner dimension (conv)
    int32_t kp;       // window lead: 64 * nch - 16 (conv)
    int32_t ring_waves;  // waves sharing one staging ring: 4 or 1 (conv)
    int32_t in_lo, in_hi;  // declared input range [in_lo, in_hi]
    int32_t steps;    // conv tile steps (or streaming positions / 256) per block
    int32_t ring;     // positions per LDS digit-plane ring: 256 * ring_waves + kp (conv)
    int32_t acc16;    // 1: every acc_s + 256 acc_{s+1} fits in int32 (conv); split
                      // words: every field's whole digit sum fits in int32
    int32_t dma;      // 1: next-step inputs are prefetched into LDS (conv)
    int32_t skip;     // slot whose operation is not run (the lost stream), or -1
    int32_t kind;     // convolution kernel: 0 linear, 1 circular (length n), 2 cross-correlation
    int32_t out32;    // 1: 32-bit words (w = 32): outputs stored as int32
    int32_t pad_;
    int64_t n, K, n_out;
    int64_t scalar;
    // Inputs and outputs in slot order. Slot t of an entangled group is
    // stream (r + 1 + t) mod M, so that slot t entangles with slot t - 1
    // (slot 0 with slot M - 1, stream r), slots 0 .. M-2 are the M-1 streams
    // recovery reads and the lost stream, if any, is slot M - 1. In the other
    // modes slot t is stream t (slot M: the checksum, which has no pointer).
    const int32_t *c[kFusedMaxM];
    const int32_t *operand;
    int64_t *out[kFusedMaxM];  // int32 storage when out32
    uint64_t *acc;    // inner product: kMaxSlots accumulators
    int32_t *rows;    // permutation: the streams interleaved, one row of 4 (<= 4 slots)
                      // or 8 int32 per position, in the plan's workspace
    // Single launch: completion counters of this group's work items, zero
    // between runs ([0]: layout items of a permutation, or the items of an
    // inner product; [1]: the gather items of a permutation), and the
    // counts they reach.
    uint32_t *sync;
    int32_t nsync[2];
};

// Bytes of one copy of one tap-digit plane of the convolution kernel: the
// reversed taps Q[v] = g[kp + 15 - v], v in [0, 64 nch + 16), behind up to
// 3 bytes of alignment padding, rounded to 16 (an aligned 20-byte read at
// the last fragment stays inside).
__host__ __device__ constexpr size_t conv_tap_plane_bytes(int nch)
{
    return ((size_t)64 * nch + 16 + 3 + 15) & ~(size_t)15;
}

// LDS layouts of the convolution kernel (a variant axis):
//   0: one ring per block (4 waves), tap-digit planes in 4 copies (one per
//      byte alignment: every operand fragment is four aligned words);
//   1: one ring per wave, tap planes in 4 copies;
//   2: one ring per block, tap planes in one copy (a quarter of the LDS; each
//      fragment is realigned from five words in registers), for kernels
//      whose windows leave no room for 4 copies.
constexpr int kConvLayouts = 3;
__host__ __device__ constexpr int conv_layout_waves(int layout) { return layout == 1 ? 1 : 4; }
__host__ __device__ constexpr int conv_layout_copies(int layout) { return layout == 2 ? 1 : 4; }

// LDS bytes of the convolution kernel's tap planes and chunk mask.
__host__ __device__ constexpr size_t conv_tap_lds(int nch, int lb, int copies)
{
    return (size_t)copies * lb * conv_tap_plane_bytes(nch) + 16;
}

struct Item {
    uint32_t g;       // group index
    uint32_t strip;   // strip index within the group
};

// One fused convolution kernel variant (fused_conv.hip, compiled once per
// kernel class and slot count), indexed [shape][layout]: shape 0 plain
// digits, 1 the taps' top digit sparse, 2 data words split into two fields
// (conv_shape); layout as above. Null where no group needs the variant.
constexpr int kConvShapeCount = 3;
struct ConvKernel {
    void (*launch[kConvShapeCount][kConvLayouts])(const GroupDev *g, const Item *items,
                                                  uint32_t nitems, uint32_t *flags, size_t lds,
                                                  hipStream_t s);
    hipError_t (*prepare[kConvShapeCount][kConvLayouts])(size_t lds);  // raises the LDS limit
    hipError_t (*attributes[kConvShapeCount][kConvLayouts])(hipFuncAttributes *a);  // loaded kernel
};
// The variant for (kernel class, slots, LA, LB), or null if none is built.
const ConvKernel *conv_kernel(int kclass, int slots, int la, int lb);

// A work item of the single launch: what to run (kind) on which strip of
// which group. kind: bits 0-1 category (0 convolution, 1 element-wise,
// 2 permutation layout pass), 2-5 slots, 6-9 operation, 10-13 LA, 14-16 LB,
// 17-18 shape, 19-20 LDS layout. steps: a layout item's 1024-position steps.
struct alignas(16) Task {
    uint32_t kind, g, strip, steps;
};
constexpr int kSingleLayoutSteps = 64;  // 64K positions per layout item of the single launch
constexpr int kSingleMinSteps = 4;      // shortest strip of a single-launch item, in steps
// Positions per lane and step of the element-wise kernel of an operation:
// gathers and inner products take twice stream_positions (more loads in
// flight: their loads are random rows, or they accumulate instead of store).
__host__ __device__ constexpr int stream_positions_of(int op, int slots)
{
    return stream_positions(slots) * ((op == NE_OP_INNER || op == NE_OP_PERM) ? 2 : 1);
}
enum TaskCategory : uint32_t { kTaskConv = 0, kTaskStream = 1, kTaskLayout = 2 };
__host__ __device__ constexpr uint32_t task_kind(uint32_t cat, int slots, int op, int la, int lb,
                                                 int shape, int layout)
{
    return cat | (uint32_t)slots << 2 | (uint32_t)op << 6 | (uint32_t)la << 10 |
           (uint32_t)lb << 14 | (uint32_t)shape << 17 | (uint32_t)layout << 19;
}

// The single-launch kernel of one kernel class (fused_single.hip).
struct SingleKernel {
    void (*launch)(const GroupDev *g, const Task *tasks, uint32_t ntasks, uint32_t *queue,
                   uint32_t *flags, uint32_t grid, size_t lds, hipStream_t s);
    hipError_t (*prepare)(size_t lds);                   // raises the LDS limit
    hipError_t (*blocks_per_cu)(size_t lds, int *blocks);  // resident blocks per CU
};
// Null if the class has no single-launch kernel.
const SingleKernel *single_kernel(int kclass);

// One element-wise kernel variant (fused_stream.hip, compiled once per kernel
// class): operation x slot count.
using StreamLaunch = void (*)(const GroupDev *g, const Item *items, uint32_t nitems,
                              uint32_t *flags, hipStream_t s);
// The variant for (operation, kernel class, slots), or null if none is built.
StreamLaunch stream_kernel(int op, int kclass, int slots);
void fused_interleave_launch(int cls, const GroupDev *g, const Item *items, uint32_t nitems,
                             hipStream_t s);
void fused_inner_finalize(const GroupDev *g, const uint32_t *gidx, uint32_t count,
                          uint32_t *flags, hipStream_t s);

}  // namespace ne
