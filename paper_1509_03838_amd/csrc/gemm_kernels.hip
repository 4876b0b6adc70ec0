// Fused entangled integer matrix product, one kernel class per translation
// unit (-DNE_KCLASS=k): D_m = C_m G for M blocks C_m (N x P) and a shared
// kernel matrix G (P x Q), the multiplication operator of eq. (2) applied to
// blocks of the streams (Sec. IV's GEMM case).
//
// A block computes a 32 x 32 tile of every output block (each wave a 16 x 16
// tile), streaming the inner dimension in chunks of 64:
//   * the C rows of the tile are read once as int32, entangled on load
//     (eq. (14)-(15): slot t with slot t - 1) and split into LA balanced
//     base-256 digits, written to LDS digit planes [slot][digit][row][k];
//     the checksum class stages the plain rows and their sum instead;
//   * the G columns of the tile are split into LB digits, stored transposed
//     [digit][column][k], so a lane's operand fragment (16 consecutive k of
//     one column) is one aligned 16-byte read;
//   * every digit pair (a, b) with a + b < 8 is one v_mfma_i32_16x16x64_i8
//     into the accumulator of weight a + b, exact in int32 (the host bounds
//     P); the lost slot's products are not issued.
// After the last chunk each slot's tile is recombined in 64-bit wrap-around
// arithmetic (exact modulo 2^64) and the outputs are recovered in registers
// from the M - 1 other slots (64-bit form of eq. (16)-(19)), as in the
// fused convolution, then stored as int64.
#include <limits.h>

#include "conv_variants.h"
#include "fused_kernels.h"
#include "gemm.h"

#if !defined(NE_KCLASS)
#error "NE_KCLASS selects the kernel class of this translation unit"
#endif

#define NE_CAT2(a, b) a##b
#define NE_NAME(a, b) NE_CAT2(a, b)

namespace ne {
namespace fk {

// 8 consecutive values of one C row (0 outside the matrix).
__device__ __forceinline__ void load_row8(const int32_t *src, bool full, bool vec, int64_t row_ok,
                                          int64_t kleft, int32_t (&v)[8])
{
    if (row_ok && full && vec) {
        const v4i a = load_in4(src), b = load_in4(src + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (row_ok && i < kleft) ? load_in1(src + i) : 0;
    }
}

// 8 values into L digit planes: plane a receives the 8 digit bytes of
// weight 256^a at dst + a * stride (two aligned words).
// u[i]: the L digit bytes of value i plus 0x80 each (value + digit offset,
// or the packed fields of a split word).
template <int L>
__device__ __forceinline__ void put_bytes8(const uint64_t (&u)[8], unsigned char *dst, size_t stride)
{
    uint32_t lo[8], hi[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        lo[i] = (uint32_t)u[i];
        hi[i] = (uint32_t)(u[i] >> 32);
    }
    uint32_t w0[8], w1[8];
    transpose4(lo, w0);
    transpose4(lo + 4, w1);
    if (L > 4) {
        transpose4(hi, w0 + 4);
        transpose4(hi + 4, w1 + 4);
    }
#pragma unroll
    for (int a = 0; a < L; ++a) {
        uint2 w;
        w.x = w0[a] ^ 0x80808080u;
        w.y = w1[a] ^ 0x80808080u;
        *reinterpret_cast<uint2 *>(dst + a * stride) = w;
    }
}

template <int L>
__device__ __forceinline__ void put_digits8(const int64_t (&x)[8], unsigned char *dst, size_t stride)
{
    constexpr uint64_t C = digit_offset<L>();
    uint64_t u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = (uint64_t)x[i] + C;
    put_bytes8<L>(u, dst, stride);
}

// Split words (FS digits per field): the fields of c + 2^l c' (c' = 0 for
// raw values) without forming the word -- lo = c's low l bits sign-extended,
// hi = c' + (c - lo) / 2^l -- cut into FS digits each (planes 0 .. FS-1 the
// low field, FS .. 2 FS - 1 the high one).
template <int FS>
__device__ __forceinline__ void put_fields8(const int32_t (&cur)[8], const int32_t (&prev)[8],
                                            bool entangled, int l, unsigned char *dst,
                                            size_t stride)
{
    constexpr uint32_t CF = (uint32_t)digit_offset<FS>();
    uint64_t u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int32_t lo = __builtin_amdgcn_sbfe(cur[i], 0, l);
        const int32_t cp = entangled ? prev[i] : 0;
        const int32_t hi = (int32_t)((uint32_t)cp +
                                     (uint32_t)((int32_t)((uint32_t)cur[i] - (uint32_t)lo) >> l));
        u[i] = pack_fields<FS>((uint32_t)lo + CF, (uint32_t)hi + CF);
    }
    put_bytes8<2 * FS>(u, dst, stride);
}

// FS > 0: words split at bit l into two fields of FS digits (LA = 2 FS;
// entangled and plain-same classes): planes 0 .. FS-1 hold the low field,
// FS .. LA-1 the high one, and every pair accumulates into its field's
// weight; y = lo-sum + 2^l hi-sum.
template <int LA, int LB, int NS, int KCLASS, int FS = 0>
__global__ __launch_bounds__(kBlock) void k_gemm_fused(const GemmArgs args)
{
    constexpr int mode = KCLASS == 0 ? kEntangled : (KCLASS == 2 ? kChecksum : kPlain);
    constexpr int M = KCLASS == 2 ? NS - 1 : NS;  // data blocks
    static_assert(FS == 0 || (2 * FS == LA && KCLASS != 2), "split words");
    constexpr int SL = FS + LB - 1;
    constexpr int S = FS ? 2 * SL : ((LA + LB - 1) < 8 ? (LA + LB - 1) : 8);
    constexpr int T = kGemmTile, R = kGemmRow;
    constexpr int PLANE = T * R;  // bytes of one digit plane of the tile
    static_assert(M >= 1 && M <= kFusedMaxM, "slot count");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    unsigned char *sa = smem;                                // [slot][digit][row][k]
    unsigned char *sb = smem + (size_t)NS * LA * PLANE;      // [digit][column][k]
    const GroupDev *G = &args.g;
    const int64_t N = args.N, P = args.P, Q = args.Q;
    const int skip = G->skip, l = G->l;
    const bool vec = args.vec != 0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * T, c0 = (int64_t)blockIdx.x * T;
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;  // this wave's tile in the block's
    // Staging: C row ar (8 consecutive k from ak), G column bc (8 k from bk).
    const int ar = tid >> 3, ak = (tid & 7) * 8;
    const int bc = tid & 31, bk = (tid >> 5) * 8;
    const int64_t arow = r0 + ar, bcol = c0 + bc;
    const bool arow_ok = arow < N, bcol_ok = bcol < Q;
    // Fragments: lane (i, h) reads row i (A) or column i (B), k = 16h .. 16h + 15.
    const int fi = lane & 15, fh = lane >> 4;
    uint32_t flag = 0;
    Bounds bd;

    v4i acc[NS][S];
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
        for (int s = 0; s < S; ++s) acc[t][s] = v4i{0, 0, 0, 0};

    for (int64_t kc = 0; kc < P; kc += kGemmK) {
        const int64_t kleft = P - kc - ak;  // valid k of this thread's C values
        const bool full = kleft >= 8;
        if (kc > 0) __syncthreads();  // every wave is done with the previous chunk's planes

        // C rows: entangled slot t = c_t + 2^l c_{t-1} (slot order), so only
        // the current and the previous block's values are held at a time.
        {
            int32_t prev[8], cur[8];
            int32_t sum[8];
            if (mode == kEntangled)
                load_row8(G->c[M - 1] + arow * P + kc + ak, full, vec, arow_ok, kleft, prev);
#pragma unroll
            for (int i = 0; i < 8; ++i) sum[i] = 0;
#pragma unroll
            for (int t = 0; t < M; ++t) {
                load_row8(G->c[t] + arow * P + kc + ak, full, vec, arow_ok, kleft, cur);
#pragma unroll
                for (int i = 0; i < 8; i += 2) bd.add2(cur[i], cur[i + 1]);
                if constexpr (FS > 0) {
                    if (t != skip)
                        put_fields8<FS>(cur, prev, mode == kEntangled, l,
                                        sa + ((size_t)t * LA * T + ar) * R + ak, PLANE);
                } else if (t != skip || mode == kEntangled) {
                    int64_t x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        if (mode == kEntangled)
                            x[i] = ent(cur[i], prev[i], l);
                        else
                            x[i] = cur[i];
                        if (mode == kChecksum) sum[i] += cur[i];
                    }
                    if (t != skip)
                        put_digits8<LA>(x, sa + ((size_t)t * LA * T + ar) * R + ak, PLANE);
                } else if (mode == kChecksum) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) sum[i] += cur[i];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) prev[i] = cur[i];
            }
            if (mode == kChecksum) {
                int64_t x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = sum[i];
                put_digits8<LA>(x, sa + ((size_t)M * LA * T + ar) * R + ak, PLANE);
            }
        }
        // G columns, transposed.
        {
            int64_t x[8];
            const int32_t *gp = args.g.operand + (kc + bk) * Q + bcol;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t v = (bcol_ok && kc + bk + i < P) ? load_in1(gp + (int64_t)i * Q) : 0;
                bd.add(v);
                x[i] = v;
            }
            put_digits8<LB>(x, sb + (size_t)bc * R + bk, PLANE);
        }
        __syncthreads();  // the chunk's digit planes are complete

        v4i bf[LB];
#pragma unroll
        for (int b = 0; b < LB; ++b)
            bf[b] = *reinterpret_cast<const v4i *>(sb + (size_t)b * PLANE + (wc + fi) * R + 16 * fh);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (t == skip) continue;
            v4i af[LA];
#pragma unroll
            for (int a = 0; a < LA; ++a)
                af[a] = *reinterpret_cast<const v4i *>(sa + (size_t)(t * LA + a) * PLANE +
                                                       (wr + fi) * R + 16 * fh);
#pragma unroll
            for (int b = 0; b < LB; ++b)
#pragma unroll
                for (int a = 0; a < LA; ++a)
                    if (pair_runs<FS>(a, b))
                        acc[t][acc_of<FS, LB>(a) + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            af[a], bf[b], acc[t][acc_of<FS, LB>(a) + b], 0, 0, 0);
        }
    }

    // y = sum_s 256^s acc_s (mod 2^64), per slot; lane (i, h) holds rows
    // 4h .. 4h + 3 of column i of its wave's tile.
    int64_t dl[NS][4];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if constexpr (FS > 0) {
                uint64_t ylo = (uint64_t)(int64_t)acc[t][SL - 1][v];
                uint64_t yhi = (uint64_t)(int64_t)acc[t][S - 1][v];
#pragma unroll
                for (int s = SL - 2; s >= 0; --s) {
                    ylo = (ylo << 8) + (uint64_t)(int64_t)acc[t][s][v];
                    yhi = (yhi << 8) + (uint64_t)(int64_t)acc[t][SL + s][v];
                }
                dl[t][v] = (int64_t)(ylo + (yhi << l));
            } else {
                uint64_t y = (uint64_t)(int64_t)acc[t][S - 1][v];
#pragma unroll
                for (int s = S - 2; s >= 0; --s) y = (y << 8) + (uint64_t)(int64_t)acc[t][s][v];
                dl[t][v] = (int64_t)y;
            }
        }
    }
    const int64_t orow = r0 + wr + 4 * fh, ocol = c0 + wc + fi;
    int loc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        loc[v] = (orow + v < N && ocol < Q) ? (int)((4 * fh + v) * Q + fi) : INT_MAX;
    epilogue<NS, 4>(G, mode, M, skip, l, (r0 + wr) * Q + c0 + wc, INT_MAX, loc, dl, flag);
    if (bd.lo < G->in_lo || bd.hi > G->in_hi) flag |= kFlagInputRange;
    if (flag && args.flags) atomicOr(args.flags, flag);
}

// ---------------------------------------------------------- two phases
//
// Phase 1: the digit planes of every slot's value (entangled, plain, or the
// checksum sum) for all Np x Pp positions (zero outside the matrix); the
// lost slot's planes are not written (never read).
template <int LA, int NS, int KCLASS, int FS = 0>
__global__ __launch_bounds__(kBlock) void k_gemm_split_a(const GemmArgs args, GemmSplit w)
{
    static_assert(FS == 0 || (2 * FS == LA && KCLASS != 2), "split words");
    constexpr int mode = KCLASS == 0 ? kEntangled : (KCLASS == 2 ? kChecksum : kPlain);
    constexpr int M = KCLASS == 2 ? NS - 1 : NS;
    const GroupDev *G = &args.g;
    const int64_t N = args.N, P = args.P, Pp = w.Pp;
    const int skip = G->skip, l = G->l;
    const bool vec = args.vec != 0;
    const size_t plane = (size_t)w.Np * Pp;
    const int64_t kgs = Pp / 8, total = w.Np * kgs;
    Bounds bd;
    for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * kBlock) {
        const int64_t row = it / kgs, k0 = (it - row * kgs) * 8;
        const bool row_ok = row < N;
        const int64_t kleft = P - k0;
        const bool full = kleft >= 8;
        int32_t prev[8], cur[8], sum[8];
        if (mode == kEntangled) load_row8(G->c[M - 1] + row * P + k0, full, vec, row_ok, kleft, prev);
#pragma unroll
        for (int i = 0; i < 8; ++i) sum[i] = 0;
#pragma unroll
        for (int t = 0; t < M; ++t) {
            load_row8(G->c[t] + row * P + k0, full, vec, row_ok, kleft, cur);
#pragma unroll
            for (int i = 0; i < 8; i += 2) bd.add2(cur[i], cur[i + 1]);
            if (t != skip) {
                unsigned char *dst = w.a + (size_t)t * LA * plane + row * Pp + k0;
                if constexpr (FS > 0) {
                    put_fields8<FS>(cur, prev, mode == kEntangled, l, dst, plane);
                } else {
                    int64_t x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        x[i] = mode == kEntangled ? ent(cur[i], prev[i], l) : cur[i];
                    put_digits8<LA>(x, dst, plane);
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sum[i] += cur[i];
                prev[i] = cur[i];
            }
        }
        if (mode == kChecksum) {
            int64_t x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = sum[i];
            put_digits8<LA>(x, w.a + (size_t)M * LA * plane + row * Pp + k0, plane);
        }
    }
    if ((bd.lo < G->in_lo || bd.hi > G->in_hi) && args.flags) atomicOr(args.flags, kFlagInputRange);
}

// Phase 1: the digit planes of G, transposed ([digit][column][k]); lanes
// take consecutive columns so that the reads of a row of G coalesce.
template <int LB>
__global__ __launch_bounds__(kBlock) void k_gemm_split_b(const GemmArgs args, GemmSplit w)
{
    const GroupDev *G = &args.g;
    const int64_t P = args.P, Q = args.Q, Pp = w.Pp, Qp = w.Qp;
    const size_t plane = (size_t)Qp * Pp;
    const int64_t total = Qp * (Pp / 8);
    Bounds bd;
    for (int64_t it = (int64_t)blockIdx.x * kBlock + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * kBlock) {
        const int64_t k0 = (it / Qp) * 8, col = it - (it / Qp) * Qp;
        int64_t x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int32_t v = (col < Q && k0 + i < P) ? load_in1(G->operand + (k0 + i) * Q + col) : 0;
            bd.add(v);
            x[i] = v;
        }
        put_digits8<LB>(x, w.b + col * Pp + k0, plane);
    }
    if ((bd.lo < G->in_lo || bd.hi > G->in_hi) && args.flags) atomicOr(args.flags, kFlagInputRange);
}

}  // namespace fk

namespace {

unsigned grid_of(int64_t items)
{
    const int64_t g = (items + fk::kBlock - 1) / fk::kBlock;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Phase 1 of the two-phase form: the digit planes of every slot and of G.
template <int LA, int LB, int NS, int FS = 0>
hipError_t launch_split(const GemmArgs &a, const GemmSplit &w, hipStream_t s)
{
    hipLaunchKernelGGL((fk::k_gemm_split_a<LA, NS, NE_KCLASS, FS>), dim3(grid_of(w.Np * (w.Pp / 8))),
                       dim3(fk::kBlock), 0, s, a, w);
    hipLaunchKernelGGL((fk::k_gemm_split_b<LB>), dim3(grid_of(w.Qp * (w.Pp / 8))), dim3(fk::kBlock),
                       0, s, a, w);
    return hipGetLastError();
}

template <int LA, int LB, int NS, int FS = 0>
hipError_t launch_one(const GemmArgs &a, hipStream_t s)
{
    void (*k)(const GemmArgs) = &fk::k_gemm_fused<LA, LB, NS, NE_KCLASS, FS>;
    const size_t lds = gemm_lds(NS, LA, LB);
    if (lds > 64 * 1024) {
        static const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((a.Q + kGemmTile - 1) / kGemmTile),
                    (unsigned)((a.N + kGemmTile - 1) / kGemmTile));
    hipLaunchKernelGGL(k, grid, dim3(fk::kBlock), lds, s, a);
    return hipGetLastError();
}

template <int LA, int LB, int NS>
constexpr GemmKernel launcher()
{
    constexpr bool conv = digits_needed(NE_KCLASS, NS, LA, LB, kGemmMaxBits) &&
                          gemm_lds(NS, LA, LB) <= 160 * 1024;
    constexpr bool split = LA % 2 == 0 && gemm_split_needed(NE_KCLASS, NS, LA, LB, kGemmMaxBits);
    GemmSplitLaunch sf = nullptr;
    GemmLaunch ff = nullptr;
    if constexpr (split) {
        sf = &launch_split<LA, LB, NS, LA / 2>;
        if constexpr (gemm_lds(NS, LA, LB) <= 160 * 1024) ff = &launch_one<LA, LB, NS, LA / 2>;
    }
    if constexpr (conv)
        return GemmKernel{&launch_one<LA, LB, NS>, &launch_split<LA, LB, NS>, sf, ff};
    else
        return GemmKernel{nullptr, nullptr, sf, ff};
}

template <int NS>
struct Row {
    GemmKernel f[kLimbsA][3];
};

template <int NS, int LA>
constexpr void fill_la(Row<NS> &r)
{
    r.f[LA - 1][0] = launcher<LA, 1, NS>();
    r.f[LA - 1][1] = launcher<LA, 2, NS>();
    r.f[LA - 1][2] = launcher<LA, 3, NS>();
}

template <int NS>
constexpr Row<NS> row()
{
    Row<NS> r{};
    fill_la<NS, 1>(r);
    fill_la<NS, 2>(r);
    fill_la<NS, 3>(r);
    fill_la<NS, 4>(r);
    fill_la<NS, 5>(r);
    fill_la<NS, 6>(r);
    fill_la<NS, 7>(r);
    fill_la<NS, 8>(r);
    return r;
}

template <int NS>
const GemmKernel *pick(int la, int lb)
{
    static constexpr Row<NS> r = row<NS>();
    const GemmKernel *k = &r.f[la - 1][lb - 1];
    return (k->fused || k->split_fields || k->fused_fields) ? k : nullptr;
}

}  // namespace

const GemmKernel *NE_NAME(gemm_kernel_, NE_KCLASS)(int slots, int la, int lb)
{
    if (la < 1 || la > kLimbsA || lb < 1 || lb > 3) return nullptr;
    switch (slots) {
    case 1: return pick<1>(la, lb);
    case 2: return pick<2>(la, lb);
    case 3: return pick<3>(la, lb);
    case 4: return pick<4>(la, lb);
    case 5: return pick<5>(la, lb);
    case 6: return pick<6>(la, lb);
    case 7: return pick<7>(la, lb);
    case 8: return pick<8>(la, lb);
    case 9: return pick<9>(la, lb);
    default: return nullptr;
    }
}

}  // namespace ne
