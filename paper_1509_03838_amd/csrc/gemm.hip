// C-ABI of the entangled integer matrix product (ne_gemm): validation, the
// range check, digit counts, the slot-order descriptor and dispatch to the
// kernel variant of gemm_kernels.hip.
#include <algorithm>

#include "conv_variants.h"
#include "gemm.h"
#include "ne_internal.h"

namespace ne {
GemmLaunch gemm_kernel_0(int slots, int la, int lb);
GemmLaunch gemm_kernel_1(int slots, int la, int lb);
GemmLaunch gemm_kernel_2(int slots, int la, int lb);

GemmLaunch gemm_kernel(int kclass, int slots, int la, int lb)
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

extern "C" ne_status ne_gemm(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q,
                             const int32_t *const *c, const int32_t *g, int64_t *const *out,
                             int32_t lost, int32_t in_bits, uint32_t *flags, ne_stream stream)
{
    if (mode < kEntangled || mode > kChecksum) return NE_EINVAL;
    const int minM = mode == kEntangled ? 3 : (mode == kChecksum ? 2 : 1);
    if (M < minM || M > kFusedMaxM || N < 0 || P < 0 || Q < 0 || !c || !out) return NE_EINVAL;
    if (in_bits < 1 || in_bits > 32) return NE_EINVAL;
    if (lost < -1 || lost >= M) return NE_EFAILIDX;
    if (in_bits > kGemmMaxBits) return NE_EUNSUP;
    if (N > (int64_t)kGemmTile * 65535 || Q > ((int64_t)1 << 26) || P > ((int64_t)1 << 24))
        return NE_EUNSUP;
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
    const DigitCounts dc = conv_digits(mode, M, in_bits);
    // int32 accumulation: a digit product is at most 2^14, summed over the
    // padded inner dimension and at most min(la, lb) pairs per weight.
    const int64_t pp = (P + kGemmK - 1) / kGemmK * kGemmK;
    if (pp * std::min(dc.la, dc.lb) * 16384 >= ((int64_t)1 << 31)) return NE_EUNSUP;
    const int nslots = mode == kChecksum ? M + 1 : M;
    const GemmLaunch launch = gemm_kernel(conv_class_of_mode(mode), nslots, dc.la, dc.lb);
    if (!launch) return NE_EUNSUP;

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
    const hipError_t e = launch(a, (hipStream_t)stream);
    return e == hipSuccess ? NE_OK : hip_fail(e);
}
