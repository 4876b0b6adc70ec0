// Fused batched kernels: for every group of M streams, entangle on load
// (eq. (14)-(15)), run the LSB operation on each entangled stream (eq. (9)),
// and recover every output from M-1 of them (eq. (16)-(19)) -- in one pass
// over HBM: the inputs are read once as int32 and only the recovered int64
// outputs are written. The entangled words and the entangled outputs live in
// LDS and registers only.
//
// Convolution runs on the i8 matrix cores as a Toeplitz product. A block
// step covers 1024 consecutive outputs; wave w owns the 16x16 tile of
// outputs y[T + 256w + 16i + j] (row i, column j), and
//     y[P + 16i + j] = sum_s A[i][s] B[s][j],
//     A[i][s] = x[P + 16i - kp + s],  B[s][j] = g[j + kp - s]  (0 outside [0, K)),
// with s over 64*nch >= K + 15 values and kp = 64*nch - 16, so every row of
// A is a contiguous window of the stream: the staged window of the block is
// the whole A operand. Words are split into balanced base-256 digits in
// [-128, 127] (LA digits for data words, LB for taps); every digit pair is
// one v_mfma_i32_16x16x64_i8 with exact int32 accumulation, and
// y = sum 256^(a+b) acc_ab is recombined in 64-bit wrap-around arithmetic,
// which is exact modulo 2^64 whatever the digit count (a word that needs more
// digits than chosen is flagged, never silently truncated).
//
// Every stream's entangled output depends only on its own entangled input;
// the stream the plan marks as lost is simply not computed, and recovery
// never reads its slot.
#include "fused.h"
#include "ne_internal.h"

namespace ne {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

// ------------------------------------------------------------- helpers

// Maps blockIdx to a work item so that each XCD (blocks are dealt to the 8
// XCDs round-robin) receives a contiguous run of items: neighbouring strips
// of a stream share their halo through that XCD's L2.
__device__ __forceinline__ uint32_t item_index(uint32_t nitems)
{
    const uint32_t per = (nitems + 7u) >> 3;
    return (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

// Balanced base-256 digits of x: x = sum_a d[a] 256^a (mod 2^64), each
// d[a] in [-128, 127]. Returns whether the digits are exact (always, modulo
// 2^64, when L = 8).
template <int L>
__device__ __forceinline__ bool split_digits(int64_t x, int32_t (&d)[L])
{
    int64_t v = x;
#pragma unroll
    for (int a = 0; a < L; ++a) {
        const int32_t di = (int32_t)(int8_t)(uint8_t)(uint64_t)v;
        d[a] = di;
        v = (int64_t)((uint64_t)v - (uint64_t)(int64_t)di) >> 8;
    }
    return L >= 8 || v == 0;
}

__device__ __forceinline__ int64_t ent(int64_t cur, int64_t prev, int l)
{
    return (int64_t)((uint64_t)cur + ((uint64_t)prev << l));
}

__device__ __forceinline__ int64_t *out_ptr(const GroupDev *G, int m) { return G->out[m]; }

// Results of one lane: V positions, one entangled (or plain) output per
// slot. Slot t of an entangled group is stream (r + 1 + t) mod M, so that
// slots 0 .. M-2 are exactly the M-1 streams recovery reads and slot M-1 is
// stream r. Slot t of the other modes is stream t (slot M: the checksum).
//
// Entangled recovery (64-bit form of eq. (16)-(19), see stream_kernels):
// d_temp's low (M-1)l bits give d_{r-1}; then d_{j-1} = (delta_j - d_j) >> l
// walking back to d_r. When stream r was not lost its slot is redundant and
// is checked against the recovered outputs instead.
template <int NS, int V>
__device__ __forceinline__ void epilogue(const GroupDev *G, int mode, int M, int r, int lost, int l,
                                         int64_t n_out, const int64_t (&dl)[NS][V],
                                         const int64_t (&pos)[V], uint32_t &flag)
{
    if (mode == kEntangled) {
        const int s = 64 - (M - 1) * l;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool ok = pos[v] < n_out;
            uint64_t acc = 0;
#pragma unroll
            for (int t = 0; t < NS - 1; ++t) {
                if (t < M - 1) {
                    const uint64_t x = (uint64_t)dl[t][v];
                    acc = (acc << l) + (((M + t) & 1) ? (uint64_t)0 - x : x);
                }
            }
            int64_t cur = ((int64_t)(acc << s)) >> s;  // d_{r-1}
            const int64_t d_prev = cur;
            if (ok) out_ptr(G, (r + M - 1) % M)[pos[v]] = cur;
#pragma unroll
            for (int t = NS - 2; t >= 0; --t) {
                if (t <= M - 2) {
                    cur = (int64_t)((uint64_t)dl[t][v] - (uint64_t)cur) >> l;
                    const int m = (t == 0) ? r : (r + t) % M;
                    if (ok) out_ptr(G, m)[pos[v]] = cur;
                }
            }
            // cur is d_r; with stream r computed, delta_r = d_r + 2^l d_{r-1}
            if (!lost && ok) {
                int64_t dr_slot = 0;
#pragma unroll
                for (int t = 0; t < NS; ++t)
                    if (t == M - 1) dr_slot = dl[t][v];
                if ((uint64_t)dr_slot != (uint64_t)cur + ((uint64_t)d_prev << l)) flag |= kFlagMismatch;
            }
        }
    } else if (mode == kChecksum) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (pos[v] >= n_out) continue;
            uint64_t e = 0, sum = 0;
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t == M) e = (uint64_t)dl[t][v];
#pragma unroll
            for (int t = 0; t < NS - 1; ++t)
                if (t < M && !(lost && t == r)) {
                    sum += (uint64_t)dl[t][v];
                    out_ptr(G, t)[pos[v]] = dl[t][v];
                }
            if (lost)
                out_ptr(G, r)[pos[v]] = (int64_t)(e - sum);
            else if (e != sum)
                flag |= kFlagMismatch;
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (pos[v] >= n_out) continue;
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t < M && !(lost && t == r)) out_ptr(G, t)[pos[v]] = dl[t][v];
        }
    }
}

// Stream (plane) that slot t holds.
__device__ __forceinline__ int slot_stream(int mode, int M, int r, int t)
{
    return mode == kEntangled ? (r + 1 + t) % M : t;
}

__device__ __forceinline__ bool slot_live(int mode, int M, int r, int lost, int t, int nslots)
{
    if (t >= nslots) return false;
    if (!lost) return true;
    return mode == kEntangled ? t != M - 1 : t != r;
}

// ----------------------------------------------------- convolution kernel

template <int LA, int LB, int NS>
__global__ __launch_bounds__(kBlock) void k_conv_fused(const GroupDev *__restrict__ groups,
                                                       const Item *__restrict__ items,
                                                       uint32_t nitems, uint32_t *flags)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const uint32_t ii = item_index(nitems);
    if (ii >= nitems) return;
    const Item it = items[ii];
    const GroupDev *G = groups + it.g;
    const int mode = G->mode, M = G->M, r = G->r, lost = G->lost, l = G->l;
    const int nslots = G->nslots, nch = G->nch, kp = G->kp, wlen = G->wlen;
    const int in_lo = G->in_lo, in_hi = G->in_hi, steps = G->steps;
    const int64_t n = G->n, K = G->K, n_out = G->n_out;
    const int32_t *__restrict__ g = G->operand;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nplanes = (mode == kChecksum) ? M + 1 : M;
    uint32_t flag = 0;

    v4i *bfrag = reinterpret_cast<v4i *>(smem);
    unsigned char *planes = smem + (size_t)nch * LB * 1024;

    // Toeplitz operand B, in the lane layout of the MFMA: lane (j, h) holds
    // B[64c + 16h + q][j] for q = 0..15, split into LB digit planes.
    for (int e = tid; e < nch * 64; e += kBlock) {
        const int c = e >> 6, ln = e & 63, j = ln & 15, h = ln >> 4;
        uint32_t w[LB][4];
#pragma unroll
        for (int b = 0; b < LB; ++b)
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) w[b][q4] = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t idx = (int64_t)j + kp - (64 * c + 16 * h + q);
            int32_t gv = 0;
            if (idx >= 0 && idx < K) gv = g[idx];
            if (gv < in_lo || gv > in_hi) flag |= kFlagInputRange;
            int32_t d[LB];
            if (!split_digits<LB>(gv, d)) flag |= kFlagLimbs;
#pragma unroll
            for (int b = 0; b < LB; ++b) w[b][q >> 2] |= ((uint32_t)d[b] & 0xffu) << (8 * (q & 3));
        }
#pragma unroll
        for (int b = 0; b < LB; ++b) {
            v4i v = {(int)w[b][0], (int)w[b][1], (int)w[b][2], (int)w[b][3]};
            bfrag[(c * LB + b) * 64 + ln] = v;
        }
    }

    for (int step = 0; step < steps; ++step) {
        const int64_t T = ((int64_t)it.strip * steps + step) * kConvTile;
        if (T >= n_out) break;
        __syncthreads();
        // Stage the window [T - kp, T + 1024) of every data word as LA digit
        // planes; entanglement happens here, on load.
        const int64_t wbase = T - kp;
        for (int gi = tid; gi < (wlen >> 2); gi += kBlock) {
            const int64_t p = wbase + 4 * gi;
            int32_t cv[kMaxSlots][4];
#pragma unroll
            for (int m = 0; m < kFusedMaxM; ++m) {
                if (m < M) {
                    if (p >= 0 && p + 4 <= n) {
                        const int4 q = *reinterpret_cast<const int4 *>(G->c[m] + p);
                        cv[m][0] = q.x; cv[m][1] = q.y; cv[m][2] = q.z; cv[m][3] = q.w;
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            cv[m][q] = (p + q >= 0 && p + q < n) ? G->c[m][p + q] : 0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (cv[m][q] < in_lo || cv[m][q] > in_hi) flag |= kFlagInputRange;
                }
            }
#pragma unroll
            for (int pl = 0; pl < kMaxSlots; ++pl) {
                if (pl >= nplanes) continue;
                uint32_t w[LA];
#pragma unroll
                for (int a = 0; a < LA; ++a) w[a] = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int64_t x = 0;
                    if (mode == kEntangled) {
#pragma unroll
                        for (int m = 0; m < kFusedMaxM; ++m)
                            if (m == pl) {
                                int32_t prev = 0;
#pragma unroll
                                for (int mm = 0; mm < kFusedMaxM; ++mm)
                                    if (mm == (m + M - 1) % M) prev = cv[mm][q];
                                x = ent(cv[m][q], prev, l);
                            }
                    } else if (pl == M) {  // checksum stream, eq. (4)
#pragma unroll
                        for (int m = 0; m < kFusedMaxM; ++m)
                            if (m < M) x += cv[m][q];
                    } else {
#pragma unroll
                        for (int m = 0; m < kFusedMaxM; ++m)
                            if (m == pl) x = cv[m][q];
                    }
                    int32_t d[LA];
                    if (!split_digits<LA>(x, d)) flag |= kFlagLimbs;
#pragma unroll
                    for (int a = 0; a < LA; ++a) w[a] |= ((uint32_t)d[a] & 0xffu) << (8 * q);
                }
#pragma unroll
                for (int a = 0; a < LA; ++a)
                    *reinterpret_cast<uint32_t *>(planes + (size_t)(pl * LA + a) * wlen + 4 * gi) = w[a];
            }
        }
        __syncthreads();

        // Each wave: its 16x16 output tile, for every live slot.
        const int64_t P0 = T + 256 * wave;
        const int aoff = 256 * wave + 16 * (lane & 15) + 16 * (lane >> 4);
        int64_t dl[NS][4];
#pragma unroll
        for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) dl[t][v] = 0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (!slot_live(mode, M, r, lost, t, nslots)) continue;
            const int pl = slot_stream(mode, M, r, t);
            const unsigned char *pbase = planes + (size_t)pl * LA * wlen + aoff;
            v4i acc[LA + LB - 1];
#pragma unroll
            for (int s = 0; s < LA + LB - 1; ++s) acc[s] = v4i{0, 0, 0, 0};
            for (int c = 0; c < nch; ++c) {
                v4i bf[LB], af[LA];
#pragma unroll
                for (int b = 0; b < LB; ++b) bf[b] = bfrag[(c * LB + b) * 64 + lane];
#pragma unroll
                for (int a = 0; a < LA; ++a)
                    af[a] = *reinterpret_cast<const v4i *>(pbase + (size_t)a * wlen + 64 * c);
                // A digit pair with a + b >= 8 is a multiple of 2^64: skipped.
#pragma unroll
                for (int b = 0; b < LB; ++b)
#pragma unroll
                    for (int a = 0; a < LA; ++a)
                        if (a + b < 8)
                            acc[a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b],
                                                                               acc[a + b], 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uint64_t y = 0;
#pragma unroll
                for (int s = 0; s < LA + LB - 1; ++s)
                    if (s < 8) y += (uint64_t)(int64_t)acc[s][v] << (8 * s);
                dl[t][v] = (int64_t)y;
            }
        }
        int64_t pos[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) pos[v] = P0 + 16 * (4 * (lane >> 4) + v) + (lane & 15);
        epilogue<NS, 4>(G, mode, M, r, lost, l, n_out, dl, pos, flag);
    }
    if (flag) atomicOr(flags, flag);
}

// ------------------------------------------------ element-wise operations

// Scale, add, permutation and inner product: one position per lane per
// step, all M streams of the group at once (entangle -> op -> recover in
// registers). Inner products accumulate per slot into the group's
// accumulators; k_inner_finalize recovers them.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_stream_fused(const GroupDev *__restrict__ groups,
                                                         const Item *__restrict__ items,
                                                         uint32_t nitems, uint32_t *flags)
{
    const uint32_t ii = item_index(nitems);
    if (ii >= nitems) return;
    const Item it = items[ii];
    const GroupDev *G = groups + it.g;
    const int op = G->op, mode = G->mode, M = G->M, r = G->r, lost = G->lost, l = G->l;
    const int nslots = G->nslots, in_lo = G->in_lo, in_hi = G->in_hi, steps = G->steps;
    const int64_t n = G->n, sv = G->scalar;
    const int32_t *__restrict__ opd = G->operand;
    uint32_t flag = 0;
    uint64_t iacc[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) iacc[t] = 0;

    const int64_t base = (int64_t)it.strip * steps * kBlock;
    for (int q = 0; q < steps; ++q) {
        const int64_t p = base + (int64_t)q * kBlock + threadIdx.x;
        if (p >= n) break;
        int64_t src = p;
        if (op == NE_OP_PERM) {
            src = opd[p];
            src = src < 0 ? 0 : (src >= n ? n - 1 : src);
        }
        int32_t cv[kFusedMaxM];
#pragma unroll
        for (int m = 0; m < kFusedMaxM; ++m) {
            cv[m] = (m < M) ? G->c[m][src] : 0;
            if (m < M && (cv[m] < in_lo || cv[m] > in_hi)) flag |= kFlagInputRange;
        }
        int32_t gv = 0;
        if (op == NE_OP_ADD || op == NE_OP_INNER) {
            gv = opd[p];
            if (gv < in_lo || gv > in_hi) flag |= kFlagInputRange;
        }
        int64_t dl[NS][1];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            dl[t][0] = 0;
            if (!slot_live(mode, M, r, lost, t, nslots)) continue;
            const int pl = slot_stream(mode, M, r, t);
            int64_t x = 0, gs = gv;
            if (mode == kEntangled) {
#pragma unroll
                for (int m = 0; m < kFusedMaxM; ++m)
                    if (m == pl) {
                        int32_t prev = 0;
#pragma unroll
                        for (int mm = 0; mm < kFusedMaxM; ++mm)
                            if (mm == (m + M - 1) % M) prev = cv[mm];
                        x = ent(cv[m], prev, l);
                    }
                gs = ent(gv, gv, l);  // footnote 3: the added vector is entangled too
            } else if (pl == M) {
#pragma unroll
                for (int m = 0; m < kFusedMaxM; ++m)
                    if (m < M) x += cv[m];
                gs = (int64_t)M * gv;  // checksum of the M added operands
            } else {
#pragma unroll
                for (int m = 0; m < kFusedMaxM; ++m)
                    if (m == pl) x = cv[m];
            }
            uint64_t y;
            switch (op) {
            case NE_OP_SCALE: y = (uint64_t)x * (uint64_t)sv; break;
            case NE_OP_ADD: y = (uint64_t)x + (uint64_t)gs; break;
            case NE_OP_INNER: y = (uint64_t)x * (uint64_t)(int64_t)gv; break;
            default: y = (uint64_t)x; break;  // permutation: the gather above
            }
            if (op == NE_OP_INNER)
                iacc[t] += y;
            else
                dl[t][0] = (int64_t)y;
        }
        if (op != NE_OP_INNER) {
            const int64_t pos[1] = {p};
            epilogue<NS, 1>(G, mode, M, r, lost, l, n, dl, pos, flag);
        }
    }
    if (op == NE_OP_INNER) {
        __shared__ uint64_t part[kBlock / 64][NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            uint64_t v = iacc[t];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                v += (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
            if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][t] = v;
        }
        __syncthreads();
        if (threadIdx.x < NS && (int)threadIdx.x < nslots) {
            uint64_t s = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += part[w][threadIdx.x];
            atomicAdd(reinterpret_cast<unsigned long long *>(G->acc + threadIdx.x),
                      (unsigned long long)s);
        }
    }
    if (flag) atomicOr(flags, flag);
}

// Recovery of inner products (one output per stream) after all partial
// sums have landed; also clears the accumulators for the next run.
template <int NS>
__global__ __launch_bounds__(64) void k_inner_finalize(const GroupDev *__restrict__ groups,
                                                       const uint32_t *__restrict__ gidx,
                                                       uint32_t count, uint32_t *flags)
{
    const uint32_t i = blockIdx.x * 64 + threadIdx.x;
    if (i >= count) return;
    const GroupDev *G = groups + gidx[i];
    uint32_t flag = 0;
    int64_t dl[NS][1];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        dl[t][0] = (int64_t)G->acc[t];
        G->acc[t] = 0;
    }
    const int64_t pos[1] = {0};
    epilogue<NS, 1>(G, G->mode, G->M, G->r, G->lost, G->l, 1, dl, pos, flag);
    if (flag) atomicOr(flags, flag);
}

}  // namespace

// ------------------------------------------------------------ launchers

using ConvLaunch = void (*)(const GroupDev *, const Item *, uint32_t, uint32_t *, size_t,
                            hipStream_t);

template <int LA, int LB, int NS>
static void conv_launch(const GroupDev *g, const Item *items, uint32_t nitems, uint32_t *flags,
                        size_t lds, hipStream_t s)
{
    const uint32_t grid = ((nitems + 7u) >> 3) << 3;
    hipLaunchKernelGGL((k_conv_fused<LA, LB, NS>), dim3(grid), dim3(kBlock), lds, s, g, items,
                       nitems, flags);
}

template <int LA, int LB, int NS>
static hipError_t conv_set_lds(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_fused<LA, LB, NS>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

#define NE_CONV_ROW(LA, NS)                                                                \
    {conv_launch<LA, 1, NS>, conv_launch<LA, 2, NS>, conv_launch<LA, 3, NS>,               \
     conv_launch<LA, 4, NS>}
#define NE_LDS_ROW(LA, NS)                                                                 \
    {conv_set_lds<LA, 1, NS>, conv_set_lds<LA, 2, NS>, conv_set_lds<LA, 3, NS>,            \
     conv_set_lds<LA, 4, NS>}

// [slot-capacity class][LA - 1][LB - 1]; class 0 holds up to 4 slots (M <= 3
// with a checksum stream, M <= 4 otherwise), class 1 up to kMaxSlots.
static const ConvLaunch kConvTable[2][kLimbsA][kLimbsB] = {
    {NE_CONV_ROW(1, 4), NE_CONV_ROW(2, 4), NE_CONV_ROW(3, 4), NE_CONV_ROW(4, 4),
     NE_CONV_ROW(5, 4), NE_CONV_ROW(6, 4), NE_CONV_ROW(7, 4), NE_CONV_ROW(8, 4)},
    {NE_CONV_ROW(1, 9), NE_CONV_ROW(2, 9), NE_CONV_ROW(3, 9), NE_CONV_ROW(4, 9),
     NE_CONV_ROW(5, 9), NE_CONV_ROW(6, 9), NE_CONV_ROW(7, 9), NE_CONV_ROW(8, 9)}};
static hipError_t (*const kLdsTable[2][kLimbsA][kLimbsB])(size_t) = {
    {NE_LDS_ROW(1, 4), NE_LDS_ROW(2, 4), NE_LDS_ROW(3, 4), NE_LDS_ROW(4, 4),
     NE_LDS_ROW(5, 4), NE_LDS_ROW(6, 4), NE_LDS_ROW(7, 4), NE_LDS_ROW(8, 4)},
    {NE_LDS_ROW(1, 9), NE_LDS_ROW(2, 9), NE_LDS_ROW(3, 9), NE_LDS_ROW(4, 9),
     NE_LDS_ROW(5, 9), NE_LDS_ROW(6, 9), NE_LDS_ROW(7, 9), NE_LDS_ROW(8, 9)}};

hipError_t fused_conv_prepare(int cls, int la, int lb, size_t lds)
{
    return kLdsTable[cls][la - 1][lb - 1](lds);
}

void fused_conv_launch(int cls, int la, int lb, const GroupDev *g, const Item *items,
                       uint32_t nitems, uint32_t *flags, size_t lds, hipStream_t s)
{
    kConvTable[cls][la - 1][lb - 1](g, items, nitems, flags, lds, s);
}

void fused_stream_launch(int cls, const GroupDev *g, const Item *items, uint32_t nitems,
                         uint32_t *flags, hipStream_t s)
{
    const uint32_t grid = ((nitems + 7u) >> 3) << 3;
    if (cls == 0)
        hipLaunchKernelGGL(k_stream_fused<4>, dim3(grid), dim3(kBlock), 0, s, g, items, nitems,
                           flags);
    else
        hipLaunchKernelGGL(k_stream_fused<kMaxSlots>, dim3(grid), dim3(kBlock), 0, s, g, items,
                           nitems, flags);
}

void fused_inner_finalize(const GroupDev *g, const uint32_t *gidx, uint32_t count,
                          uint32_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_inner_finalize<kMaxSlots>, dim3((count + 63) / 64), dim3(64), 0, s, g,
                       gidx, count, flags);
}

}  // namespace ne
