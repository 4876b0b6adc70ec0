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

// Two-phase path: the digit planes of every slot's C values and of G are
// written once to caller workspace; then every computed slot's product is
// an independent slice of one launch (blockIdx.z), each wave a 32 x 32 tile
// read straight from the planes (no staging, no barriers), written as int64
// entangled outputs into that stream's output buffer (the checksum slot's
// into workspace); recovery follows in place (the per-step extraction, or
// the checksum recovery).
constexpr int kGemmSplitRows = 64, kGemmSplitCols = 64;

struct GemmSplit {
    int64_t Np, Pp, Qp;  // N, P, Q rounded up to the block rows, 64 and the block columns
    unsigned char *a;    // slots x LA planes of Np x Pp digit bytes ([slot][digit][row][k])
    unsigned char *b;    // LB planes of Qp x Pp digit bytes ([digit][column][k])
    int64_t *e;          // checksum method: the checksum slot's N x Q products
};

inline int64_t gemm_round(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Workspace bytes of the two-phase path (256-byte aligned pieces).
inline size_t gemm_split_bytes(int slots, int la, int lb, int64_t N, int64_t P, int64_t Q,
                               bool checksum)
{
    const int64_t Np = gemm_round(N, kGemmSplitRows), Pp = gemm_round(P, kGemmK),
                  Qp = gemm_round(Q, kGemmSplitCols);
    return (size_t)gemm_round((int64_t)slots * la * Np * Pp, 256) +
           (size_t)gemm_round((int64_t)lb * Qp * Pp, 256) + (checksum ? (size_t)N * Q * 8 : 0);
}

using GemmLaunch = hipError_t (*)(const GemmArgs &a, hipStream_t s);
using GemmSplitLaunch = hipError_t (*)(const GemmArgs &a, const GemmSplit &w, hipStream_t s);
struct GemmKernel {
    GemmLaunch fused;              // one pass, digits staged in LDS
    GemmSplitLaunch split;         // two phases through workspace
    GemmSplitLaunch split_fields;  // two phases, words split into two fields of LA / 2 digits
    GemmLaunch fused_fields;       // one pass, words split into two fields of LA / 2 digits
};
// The variant for (kernel class, slots, LA, LB), or null if none is built
// (a variant may hold only the split-word phase 1).
const GemmKernel *gemm_kernel(int kclass, int slots, int la, int lb);

}  // namespace ne
