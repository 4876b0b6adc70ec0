// C-ABI of the entangled integer matrix product (ne_gemm): validation, the
// range check, digit counts, the slot-order descriptor and dispatch to the
// kernel variant of gemm_kernels.hip.
#include <algorithm>

#include "conv_variants.h"
#include "gemm.h"
#include "ne_internal.h"

namespace ne {
const GemmKernel *gemm_kernel_0(int slots, int la, int lb);
const GemmKernel *gemm_kernel_1(int slots, int la, int lb);
const GemmKernel *gemm_kernel_2(int slots, int la, int lb);

const GemmKernel *gemm_kernel(int kclass, int slots, int la, int lb)
{
    switch (kclass) {
    case 0: return gemm_kernel_0(slots, la, lb);
    case 1: return gemm_kernel_1(slots, la, lb);
    case 2: return gemm_kernel_2(slots, la, lb);
    default: return nullptr;
    }
}
}  // namespace ne

using namespace ne;

namespace {

// Argument checks and digit counts shared by the size query and the call.
ne_status gemm_shape(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q, int32_t in_bits,
                     DigitCounts *dc)
{
    if (mode < kEntangled || mode > kChecksum) return NE_EINVAL;
    const int minM = mode == kEntangled ? 3 : (mode == kChecksum ? 2 : 1);
    if (M < minM || M > kFusedMaxM || N < 0 || P < 0 || Q < 0) return NE_EINVAL;
    if (in_bits < 1 || in_bits > 32) return NE_EINVAL;
    if (in_bits > kGemmMaxBits) return NE_EUNSUP;
    if (N > (int64_t)kGemmTile * 65535 || Q > ((int64_t)1 << 26) || P > ((int64_t)1 << 24))
        return NE_EUNSUP;
    *dc = conv_digits(mode, M, in_bits);
    return NE_OK;
}

}  // namespace

extern "C" ne_status ne_gemm_workspace_size(int32_t mode, int32_t M, int64_t N, int64_t P,
                                            int64_t Q, int32_t in_bits, size_t *bytes)
{
    if (!bytes) return NE_EINVAL;
    DigitCounts dc{};
    const ne_status st = gemm_shape(mode, M, N, P, Q, in_bits, &dc);
    if (st != NE_OK) return st;
    const int nslots = mode == kChecksum ? M + 1 : M;
    *bytes = (N == 0 || Q == 0) ? 0 : gemm_split_bytes(nslots, dc.la, dc.lb, N, P, Q);
    return NE_OK;
}

extern "C" ne_status ne_gemm(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q,
                             const int32_t *const *c, const int32_t *g, int64_t *const *out,
                             int32_t lost, int32_t in_bits, void *workspace,
                             size_t workspace_bytes, uint32_t *flags, ne_stream stream)
{
    DigitCounts dc0{};
    const ne_status st0 = gemm_shape(mode, M, N, P, Q, in_bits, &dc0);
    if (st0 != NE_OK) return st0;
    if (!c || !out) return NE_EINVAL;
    if (lost < -1 || lost >= M) return NE_EFAILIDX;
    if (N == 0 || Q == 0) return NE_OK;
    for (int m = 0; m < M; ++m)
        if ((!c[m] && P > 0) || !out[m]) return NE_EINVAL;
    if (!g && P > 0) return NE_EINVAL;

    // Worst case |D[i][j]| <= P 2^(b-1) 2^(b-1) (eq. (11)/(13) bound D for
    // the method; 64 bits otherwise, M times that for the checksum block).
    const unsigned __int128 B = (unsigned __int128)1 << (in_bits - 1);
    const unsigned __int128 bound = B * B * (unsigned __int128)P;
    int32_t l = 0;
    if (mode == kEntangled) {
        int32_t ll = 0, kk = 0;
        int64_t D = 0;
        if (ne_params(M, 64, &ll, &kk, &D) != NE_OK) return NE_ERANGE;
        if (bound > (unsigned __int128)D) return NE_ERANGE;
        l = ll;
    } else {
        const unsigned __int128 chk = mode == kChecksum ? bound * (unsigned)M : bound;
        if (chk > (((unsigned __int128)1 << 63) - 1)) return NE_ERANGE;
    }
    const DigitCounts dc = dc0;
    // int32 accumulation: a digit product is at most 2^14, summed over the
    // padded inner dimension and at most min(la, lb) pairs per weight.
    const int64_t pp = (P + kGemmK - 1) / kGemmK * kGemmK;
    if (pp * std::min(dc.la, dc.lb) * 16384 >= ((int64_t)1 << 31)) return NE_EUNSUP;
    const int nslots = mode == kChecksum ? M + 1 : M;
    const GemmKernel *kern = gemm_kernel(conv_class_of_mode(mode), nslots, dc.la, dc.lb);
    if (!kern) return NE_EUNSUP;
    const size_t need = gemm_split_bytes(nslots, dc.la, dc.lb, N, P, Q);
    if (workspace && (workspace_bytes < need || (uintptr_t)workspace % 256)) return NE_EINVAL;

    GemmArgs a{};
    GroupDev &G = a.g;
    G.op = -1;
    G.M = M;
    G.mode = mode;
    G.lost = lost >= 0 ? 1 : 0;
    G.r = lost >= 0 ? lost : 0;
    G.l = l;
    G.la = dc.la;
    G.lb = dc.lb;
    G.nslots = nslots;
    G.in_lo = -(int32_t)((int64_t)1 << (in_bits - 1));
    G.in_hi = (int32_t)(((int64_t)1 << (in_bits - 1)) - 1);
    G.skip = G.lost ? (mode == kEntangled ? M - 1 : G.r) : -1;
    bool vec = (P % 4) == 0;
    for (int t = 0; t < M; ++t) {
        const int m = mode == kEntangled ? (G.r + 1 + t) % M : t;
        G.c[t] = c[m];
        G.out[t] = out[m];
        if ((uintptr_t)c[m] % 16) vec = false;
    }
    G.operand = g;
    a.N = N;
    a.P = P;
    a.Q = Q;
    a.flags = flags;
    a.vec = vec ? 1 : 0;
    hipError_t e;
    if (workspace) {
        GemmSplit w{};
        w.Np = gemm_round(N, kGemmSplitRows);
        w.Pp = gemm_round(P, kGemmK);
        w.Qp = gemm_round(Q, kGemmSplitCols);
        w.a = (unsigned char *)workspace;
        w.b = w.a + gemm_round((int64_t)(nslots * dc.la * (size_t)w.Np * w.Pp), 256);
        if (w.Qp / kGemmSplitCols > 0x7fffffff || w.Np / kGemmSplitRows > 65535) return NE_EUNSUP;
        e = kern->split(a, w, (hipStream_t)stream);
    } else {
        e = kern->fused(a, (hipStream_t)stream);
    }
    return e == hipSuccess ? NE_OK : hip_fail(e);
}
