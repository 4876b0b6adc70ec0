// Entangled integer matrix product (private to libne): the descriptor of one
// call and the kernel-variant table.
#pragma once

#include "fused.h"

namespace ne {

constexpr int kGemmTile = 32;  // outputs per block side: 4 waves of 16 x 16
constexpr int kGemmK = 64;     // inner-dimension chunk per LDS stage (one MFMA depth)
constexpr int kGemmRow = 80;   // LDS bytes per digit-plane row: 64 k + 16 (conflict-free reads)
constexpr int kGemmMaxBits = 16;  // input and kernel-matrix values of at most 16 bits

struct GemmArgs {
    GroupDev g;        // streams and outputs in slot order, M, mode, l, skip, declared range
    int64_t N, P, Q;   // C_m: N x P, G: P x Q, D_m: N x Q (row-major)
    uint32_t *flags;   // device flag word (NE_FLAG_*), or null
    int32_t vec;       // 1: every row of every C_m starts 16-byte aligned (16-byte loads)
    int32_t pad_;
};

// LDS of a block: NS x LA digit planes of the C rows, LB of the G columns.
__host__ __device__ constexpr size_t gemm_lds(int slots, int la, int lb)
{
    return (size_t)(slots * la + lb) * kGemmTile * kGemmRow;
}

using GemmLaunch = hipError_t (*)(const GemmArgs &a, hipStream_t s);
// The variant for (kernel class, slots, LA, LB), or null if none is built.
GemmLaunch gemm_kernel(int kclass, int slots, int la, int lb);

}  // namespace ne
