// C-ABI of the entangled integer matrix product (ne_gemm): validation, the
// range check, digit counts, the slot-order descriptor and dispatch to the
// kernel variant of gemm_kernels.hip.
#include <algorithm>

#include <limits.h>

#include "conv_variants.h"
#include "fused_kernels.h"
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

namespace ne {
namespace {

// The computed slots of one call: their digit planes and output buffers.
struct DigitJob {
    const unsigned char *a[kMaxSlots];
    int64_t *d[kMaxSlots];
};

typedef __attribute__((address_space(1))) const fk::v4i gcv4i_t;
typedef __attribute__((address_space(1))) int64_t gi64_t;

// The product's int64 outputs are written once: non-temporal stores (the
// plain and checksum calls measured 2-7% faster).
__device__ __forceinline__ void store_nt(int64_t *p, int64_t v)
{
    __builtin_nontemporal_store(v, (gi64_t *)p);
}

// Phase 2: slot blockIdx.z's product. The block stages each 64-deep chunk
// of its 32 WR A rows and 64 B columns (all digit planes) in LDS once, by direct
// HBM-to-LDS loads (no staging registers: 154 instead of 206 VGPRs for the
// split-word variant) into two buffers, the next chunk's loads in flight
// while this chunk's products run, one barrier per chunk (three buffers,
// two chunks ahead, measured 5-8% slower: 72 KB of LDS admit 2 blocks per
// CU, 48 KB admit 3); every wave reads its fragments
// from there: every digit pair of 16 x 64 A and 64 x 16 B fragments goes
// into the accumulator of its weight, each wave a 16 WR x 32 tile (WR x 2
// matrix-core tiles; WR = 4 reads 20 fragments per 64 products where WR = 2
// reads 12 per 32, and stages B once per 128 rows). The entangled (or plain) int64 products
// y = sum_s 256^s acc_s (mod 2^64) go to the slot's output buffer.
//
// LDS rows are 64 bytes, unpadded (a direct load fills 1 KB contiguously):
// row r keeps its 16-byte segment s at position s ^ swz(r), so that the
// fragment reads of 16 consecutive rows fall on distinct bank groups.
constexpr int kDigitRow = 64;                            // LDS bytes per staged row
constexpr int kDigitPlane = kGemmSplitRows * kDigitRow;  // 64 rows of one digit plane of a chunk
constexpr int kDigitBuffers = 2;  // loads run kDigitBuffers - 1 chunks ahead

// LDS of one block: WR / 2 times 64 A rows and 64 B columns per plane.
__host__ __device__ constexpr size_t digits_lds(int la, int lb, int wr)
{
    return (size_t)kDigitBuffers * (la * (wr / 2) + lb) * kDigitPlane;
}

__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// FS > 0: the data planes hold split words (FS digits of the low field, then
// FS of the high field, weights 256^a and 2^l 256^a): every pair accumulates
// into its field's weight and y = lo-sum + 2^l hi-sum.
template <int LA, int LB, int FS = 0, int WR = 2>
__global__ __launch_bounds__(fk::kBlock) __attribute__((amdgpu_waves_per_eu(WR / 2)))
void k_gemm_digits(const GemmSplit w, const DigitJob job,
                                                            int64_t N, int64_t Q, int l)
{
    static_assert(kGemmSplitRows == 64 && kGemmSplitCols == 64, "block tile");
    static_assert(FS == 0 || 2 * FS == LA, "split words");
    static_assert(WR == 2 || WR == 4, "wave rows");
    constexpr int SL = FS + LB - 1;
    constexpr int S = FS ? 2 * SL : ((LA + LB - 1) < 8 ? (LA + LB - 1) : 8);
    constexpr int H = WR / 2;                    // 64-row halves of the block's A rows
    constexpr int APlane = H * kDigitPlane;      // one A digit plane of a chunk
    constexpr int Buf = LA * APlane + LB * kDigitPlane;
    constexpr int NL = LA * H + LB;              // direct loads per wave and chunk
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int fi = lane & 15, fh = lane >> 4;
    const int64_t Pp = w.Pp;
    const int64_t R0 = (int64_t)blockIdx.y * (64 * H), C0 = (int64_t)blockIdx.x * kGemmSplitCols;
    const int wr = (wave >> 1) * 16 * WR, wc = (wave & 1) * 32;
    const size_t aplane = (size_t)w.Np * Pp, bplane = (size_t)w.Qp * Pp;
    // Staging: wave v fills rows 64 h + 16 v .. 64 h + 16 v + 15 of every
    // plane, one 1 KB direct load per plane and half h; its lane i lands at
    // LDS position i of that kilobyte (row 64 h + 16 v + i / 4, position
    // i % 4) and so fetches segment (i % 4) ^ swz(row) of that row
    // (swz(row) does not depend on h).
    const int sr = 16 * wave + (lane >> 2);
    const int sseg = 16 * ((lane & 3) ^ swz(sr));
    const unsigned char *ga = job.a[blockIdx.z] + (R0 + sr) * Pp + sseg;
    const unsigned char *gb = w.b + (C0 + sr) * Pp + sseg;
    typedef __attribute__((address_space(3))) void lds_t;
    auto issue = [&](int64_t c) {
        unsigned char *buf = smem + (c % kDigitBuffers) * Buf + wave * 1024;
        const int64_t kc = c * kGemmK;
#pragma unroll
        for (int a = 0; a < LA; ++a)
#pragma unroll
            for (int h = 0; h < H; ++h)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(ga + a * aplane + (int64_t)h * 64 * Pp + kc),
                    (lds_t *)(buf + a * APlane + h * kDigitPlane), 16, 0, 0);
#pragma unroll
        for (int b = 0; b < LB; ++b)
            __builtin_amdgcn_global_load_lds((const void *)(gb + b * bplane + kc),
                                             (lds_t *)(buf + LA * APlane + b * kDigitPlane), 16, 0,
                                             0);
    };
    // this lane's fragment offsets within a plane (row * 64 + swizzled segment)
    int aoff[WR], boff[2];
#pragma unroll
    for (int t = 0; t < WR; ++t) {
        const int ra = wr + 16 * t + fi;
        aoff[t] = ra * kDigitRow + 16 * (fh ^ swz(ra));
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int rb = wc + 16 * t + fi;
        boff[t] = rb * kDigitRow + 16 * (fh ^ swz(rb));
    }
    fk::v4i acc[WR][2][S];
#pragma unroll
    for (int rt = 0; rt < WR; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int s = 0; s < S; ++s) acc[rt][ct][s] = fk::v4i{0, 0, 0, 0};
    const int64_t nc = Pp / kGemmK;
    constexpr int D = kDigitBuffers - 1;  // chunks in flight ahead
    static_assert(D == 1 || D == 2, "prefetch depth");
    if (nc > 0) issue(0);
    if (D == 2 && nc > 1) issue(1);
    for (int64_t c = 0; c < nc; ++c) {
        // this wave's loads of chunk c have landed (with D = 2 those of chunk
        // c + 1 may still be in flight: NP of them), then every wave's
        if (D == 2 && c + 1 < nc)
            __builtin_amdgcn_s_waitcnt(0xF70 | NL);  // vmcnt(NL), other counters untouched
        else
            __builtin_amdgcn_s_waitcnt(0xF70);       // vmcnt(0)
        // Then the block barrier: every wave's chunk c is in LDS, and every
        // wave is done reading buffer (c + D) % (D + 1) (chunk c - 1: its reads
        // completed before its products, which precede the barrier). A bare
        // barrier: the fence of __syncthreads would also wait for chunk
        // c + 1's loads (direct loads count as pending LDS writes). The empty
        // asm statements keep the compiler from moving LDS accesses across it.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (c + D < nc) issue(c + D);
        const unsigned char *cur = smem + (c % kDigitBuffers) * Buf;
        fk::v4i af[WR][LA], bf[2][LB];
#pragma unroll
        for (int rt = 0; rt < WR; ++rt)
#pragma unroll
            for (int a = 0; a < LA; ++a)
                af[rt][a] = *reinterpret_cast<const fk::v4i *>(cur + a * APlane + aoff[rt]);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int b = 0; b < LB; ++b)
                bf[ct][b] = *reinterpret_cast<const fk::v4i *>(cur + LA * APlane + b * kDigitPlane +
                                                               boff[ct]);
#pragma unroll
        for (int rt = 0; rt < WR; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int b = 0; b < LB; ++b)
#pragma unroll
                    for (int a = 0; a < LA; ++a)
                        if (fk::pair_runs<FS>(a, b))
                            acc[rt][ct][fk::acc_of<FS, LB>(a) + b] =
                                __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                    af[rt][a], bf[ct][b], acc[rt][ct][fk::acc_of<FS, LB>(a) + b],
                                    0, 0, 0);
    }
    int64_t *d = job.d[blockIdx.z];
#pragma unroll
    for (int rt = 0; rt < WR; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int64_t col = C0 + wc + 16 * ct + fi;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = R0 + wr + 16 * rt + 4 * fh + v;
                uint64_t y;
                if constexpr (FS > 0) {
                    uint64_t ylo = (uint64_t)(int64_t)acc[rt][ct][SL - 1][v];
                    uint64_t yhi = (uint64_t)(int64_t)acc[rt][ct][S - 1][v];
#pragma unroll
                    for (int s = SL - 2; s >= 0; --s) {
                        ylo = (ylo << 8) + (uint64_t)(int64_t)acc[rt][ct][s][v];
                        yhi = (yhi << 8) + (uint64_t)(int64_t)acc[rt][ct][SL + s][v];
                    }
                    y = ylo + (yhi << l);
                } else {
                    y = (uint64_t)(int64_t)acc[rt][ct][S - 1][v];
#pragma unroll
                    for (int s = S - 2; s >= 0; --s)
                        y = (y << 8) + (uint64_t)(int64_t)acc[rt][ct][s][v];
                }
                if (row < N && col < Q) store_nt(d + row * Q + col, (int64_t)y);
            }
        }
}

using DigitLaunch = void (*)(const GemmSplit &w, const DigitJob &job, int nslots, int64_t N,
                             int64_t Q, int l, hipStream_t s);

template <int LA, int LB, int FS, int WR>
void launch_digits_wr(const GemmSplit &w, const DigitJob &job, int nslots, int64_t N, int64_t Q,
                      int l, hipStream_t s)
{
    void (*k)(const GemmSplit, const DigitJob, int64_t, int64_t, int) =
        &k_gemm_digits<LA, LB, FS, WR>;
    constexpr size_t lds = digits_lds(LA, LB, WR);
    if (lds > 64 * 1024) {
        // raised once per variant; should it fail, the launch below fails
        // too and the caller's hipGetLastError reports it
        static const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)e;
    }
    const dim3 grid((unsigned)(w.Qp / kGemmSplitCols), (unsigned)(w.Np / (32 * WR)),
                    (unsigned)nslots);
    hipLaunchKernelGGL(k, grid, dim3(fk::kBlock), lds, s, w, job, N, Q, l);
}

// 128-row blocks (WR = 4) where the padded rows divide into them and two
// blocks still fit one CU's 160 KB of LDS; 64-row blocks otherwise.
template <int LA, int LB, int FS = 0>
void launch_digits(const GemmSplit &w, const DigitJob &job, int nslots, int64_t N, int64_t Q, int l,
                   hipStream_t s)
{
    if constexpr (2 * digits_lds(LA, LB, 4) <= 160 * 1024) {
        if (w.Np % 128 == 0) return launch_digits_wr<LA, LB, FS, 4>(w, job, nslots, N, Q, l, s);
    }
    launch_digits_wr<LA, LB, FS, 2>(w, job, nslots, N, Q, l, s);
}

#define NE_DIGITS_ROW(LA) {&launch_digits<LA, 1>, &launch_digits<LA, 2>, &launch_digits<LA, 3>}
const DigitLaunch kDigits[kLimbsA][3] = {NE_DIGITS_ROW(1), NE_DIGITS_ROW(2), NE_DIGITS_ROW(3),
                                         NE_DIGITS_ROW(4), NE_DIGITS_ROW(5), NE_DIGITS_ROW(6),
                                         NE_DIGITS_ROW(7), NE_DIGITS_ROW(8)};
#undef NE_DIGITS_ROW
// split words: FS = 1..4 digits per field (LA = 2 FS)
#define NE_SPLIT_ROW(FS) \
    {&launch_digits<2 * FS, 1, FS>, &launch_digits<2 * FS, 2, FS>, &launch_digits<2 * FS, 3, FS>}
const DigitLaunch kDigitsSplit[4][3] = {NE_SPLIT_ROW(1), NE_SPLIT_ROW(2), NE_SPLIT_ROW(3),
                                        NE_SPLIT_ROW(4)};
#undef NE_SPLIT_ROW

}  // namespace
}  // namespace ne

using namespace ne;

namespace {

// Argument checks and digit counts shared by the size query and the call.
// Both forms split words into two fields where that takes fewer planes
// (entangled and plain-same).
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
    *dc = conv_digits(mode, M, in_bits, 64, mode == kEntangled || mode == kPlainSame);
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
    *bytes = (N == 0 || Q == 0) ? 0 : gemm_split_bytes(nslots, dc.la, dc.lb, N, P, Q,
                                                       mode == kChecksum);
    return NE_OK;
}

extern "C" ne_status ne_gemm(int32_t mode, int32_t M, int64_t N, int64_t P, int64_t Q,
                             const int32_t *const *c, const int32_t *g, int64_t *const *out,
                             int32_t lost, int32_t in_bits, void *workspace,
                             size_t workspace_bytes, uint32_t *flags, ne_stream stream)
{
    DigitCounts dc{};
    const ne_status st0 = gemm_shape(mode, M, N, P, Q, in_bits, &dc);
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
    const int fs = dc.split ? dc.la / 2 : 0;
    // int32 accumulation: a digit product is at most 2^14, summed over the
    // padded inner dimension and at most min(digits of a field, lb) pairs per weight.
    const int64_t pp = (P + kGemmK - 1) / kGemmK * kGemmK;
    if (pp * std::min(fs ? fs : dc.la, dc.lb) * 16384 >= ((int64_t)1 << 31)) return NE_EUNSUP;
    const int nslots = mode == kChecksum ? M + 1 : M;
    const GemmKernel *kern = gemm_kernel(conv_class_of_mode(mode), nslots, dc.la, dc.lb);
    if (!kern) return NE_EUNSUP;
    const bool have = fs ? (workspace ? kern->split_fields != nullptr : kern->fused_fields != nullptr)
                         : kern->fused != nullptr;
    if (!have) return NE_EUNSUP;
    if (fs && (fs > 4 || dc.lb > 3)) return NE_EUNSUP;
    if (fs) l = dc.l;  // the field boundary (plain-same groups too)
    const size_t need = gemm_split_bytes(nslots, dc.la, dc.lb, N, P, Q, mode == kChecksum);
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
        w.b = w.a + gemm_round((int64_t)nslots * dc.la * w.Np * w.Pp, 256);
        w.e = (int64_t *)(w.b + gemm_round((int64_t)dc.lb * w.Qp * w.Pp, 256));
        if (w.Qp / kGemmSplitCols > 0x7fffffff || w.Np / kGemmSplitRows > 65535) return NE_EUNSUP;
        hipStream_t s = (hipStream_t)stream;
        e = fs ? kern->split_fields(a, w, s) : kern->split(a, w, s);
        if (e != hipSuccess) return hip_fail(e);
        // every computed slot's product, one z slice each
        DigitJob job{};
        int nj = 0;
        const size_t slot_bytes = (size_t)dc.la * w.Np * w.Pp;
        for (int t = 0; t < nslots; ++t) {
            if (t == G.skip) continue;
            job.a[nj] = w.a + (size_t)t * slot_bytes;
            job.d[nj] = t < M ? G.out[t] : w.e;
            ++nj;
        }
        if (fs)
            kDigitsSplit[fs - 1][dc.lb - 1](w, job, nj, N, Q, l, s);
        else
            kDigits[dc.la - 1][dc.lb - 1](w, job, nj, N, Q, l, s);
        // recovery in place
        const int64_t n = N * Q;
        if (mode == kEntangled) {
            PtrsCI64 in{};
            PtrsI64 o{};
            for (int t = 0; t < M; ++t) {
                if (t < M - 1) in.p[t] = G.out[t];
                o.p[t] = G.out[t];
            }
            launch_extract(M, l, n, in, o, s);
        } else if (mode == kChecksum && G.lost) {
            PtrsCI64 d{};
            int cnt = 0;
            for (int t = 0; t < M; ++t)
                if (t != G.r) d.p[cnt++] = G.out[t];
            launch_checksum_recover(cnt, n, d, w.e, G.out[G.r], s);
        }
        e = hipGetLastError();
    } else {
        e = fs ? kern->fused_fields(a, (hipStream_t)stream) : kern->fused(a, (hipStream_t)stream);
    }
    return e == hipSuccess ? NE_OK : hip_fail(e);
}
