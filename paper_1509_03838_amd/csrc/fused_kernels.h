// Fused batched kernels (private to libne): for every group of M streams,
// entangle on load (eq. (14)-(15)), run the LSB operation on each entangled
// stream (eq. (9)), and recover every output from M-1 of them
// (eq. (16)-(19)) -- in one pass over HBM: the inputs are read once as int32
// and only the recovered int64 outputs are written. The entangled words and
// the entangled outputs live in LDS and registers only.
//
// Convolution runs on the i8 matrix cores as a Toeplitz product. Each wave
// computes 16x16 tiles of outputs y[P + 16i + j] (row i, column j):
//     y[P + 16i + j] = sum_s A[i][s] B[s][j],
//     A[i][s] = x[P + 16i - kp + s],  B[s][j] = g[j + kp - s]  (0 outside [0, K)),
// with s over 64*nch >= K + 15 values and kp = 64*nch - 16, so every row of
// A is a contiguous window of the stream, read straight from a staging ring
// in LDS. Words are split into balanced base-256 digits in [-128, 127] (LA
// digits for data words, LB for taps); every digit pair is one
// v_mfma_i32_16x16x64_i8 with exact int32 accumulation (pairs of equal weight
// a + b share an accumulator), and y = sum 256^s acc_s is recombined in
// 64-bit wrap-around arithmetic, exact modulo 2^64. The digit counts come
// from the declared input range, and every input is checked against it
// (NE_FLAG_INPUT_RANGE), so a word never needs more digits than it gets.
//
// Every stream's entangled output depends only on its own entangled input;
// the stream the plan marks as lost is simply not computed, and recovery
// never reads its slot.
#pragma once

#include "fused.h"
#include "ne_internal.h"

namespace ne {
namespace fk {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

struct alignas(16) I64x2 {
    int64_t a, b;
};

// Maps blockIdx to a work item so that each XCD (blocks are dealt to the 8
// XCDs round-robin) receives a contiguous run of items: neighbouring strips
// of a stream share their halo through that XCD's L2.
__device__ __forceinline__ uint32_t item_index(uint32_t nitems)
{
    const uint32_t per = (nitems + 7u) >> 3;
    return (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

// The thread's index in its block, as a work item's body reads it. The
// single-launch kernel runs every body inside one loop over work items:
// there each body takes the index afresh (an empty asm the optimizer cannot
// move), so that the values a body derives from it are computed inside that
// body instead of being hoisted out of the loop and kept live across all.
__device__ __forceinline__ int item_tid()
{
    int t = (int)threadIdx.x;
#if defined(NE_SINGLE_LAUNCH)
    asm volatile("" : "+v"(t));
#endif
    return t;
}

__device__ __forceinline__ int64_t ent(int64_t cur, int64_t prev, int l)
{
    return (int64_t)((uint64_t)cur + ((uint64_t)prev << l));
}

// Global-memory views of the descriptor's stream pointers (the descriptor
// holds generic pointers; global accesses take scalar base addresses and do
// not count against the LDS wait counter).
typedef __attribute__((address_space(1))) int64_t gi64_t;
typedef __attribute__((address_space(1))) const v4i gv4i_t;

typedef __attribute__((address_space(1))) int32_t gi32_t;

__device__ __forceinline__ void store_out(int64_t *p, int64_t v) { *(gi64_t *)p = v; }

// One recovered output at index idx of an output stream: int64, or int32 in
// groups of 32-bit words (the value then fits 32 bits by the plan's range
// check). The int64 stores are non-temporal: outputs are written once and not
// read again by the kernel (about 2% faster on the batched convolution); the
// int32 ones, whose 16-lane rows fill half a cache line, are not (the
// non-temporal form measured slower there).
__device__ __forceinline__ void store_out(int64_t *base, int64_t idx, int64_t v, bool o32)
{
    if (o32)
        *(gi32_t *)((int32_t *)base + idx) = (int32_t)v;
    else
        __builtin_nontemporal_store(v, (gi64_t *)(base + idx));
}
__device__ __forceinline__ v4i load_in4(const int32_t *p) { return *(gv4i_t *)p; }
__device__ __forceinline__ int32_t load_in1(const int32_t *p)
{
    return *(const __attribute__((address_space(1))) int32_t *)p;
}

// Running bounds of every input value a thread reads; checked once against
// the declared range at the end of the kernel.
struct Bounds {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    __device__ __forceinline__ void add(int32_t v)
    {
        lo = min(lo, v);
        hi = max(hi, v);
    }
    __device__ __forceinline__ void add2(int32_t a, int32_t b)
    {
        lo = min(lo, min(a, b));
        hi = max(hi, max(a, b));
    }
};

// Results of one lane: V positions base + loc[v], one entangled (or plain)
// output per slot (slot order: the descriptor's comment).
//
// Entangled recovery (64-bit form of eq. (16)-(19), as in the streaming
// extraction kernel): d_temp's low (M-1)l bits give the output of slot M-2
// (stream r - 1); then d_{t-1} = (delta_t - d_t) >> l walks back through
// slots M-3, ..., 0 to slot M-1 (stream r). When slot M-1 was computed too
// (no loss) it is redundant and is checked against the recovered outputs.
template <int NS, int V>
__device__ __forceinline__ void epilogue(const GroupDev *G, int mode, int M, int skip, int l,
                                         int64_t base, int64_t lim, const int (&loc)[V],
                                         const int64_t (&dl)[NS][V], uint32_t &flag)
{
    const bool o32 = G->out32 != 0;
    if (mode == kEntangled) {
        const int s = 64 - (M - 1) * l;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool ok = loc[v] < lim;
            const int64_t at = base + loc[v];
            uint64_t acc = 0;
#pragma unroll
            for (int t = 0; t < NS - 1; ++t) {
                if (t < M - 1) {
                    const uint64_t x = (uint64_t)dl[t][v];
                    acc = (acc << l) + (((M + t) & 1) ? (uint64_t)0 - x : x);
                }
            }
            int64_t cur = ((int64_t)(acc << s)) >> s;  // output of slot M-2
            const int64_t d_prev = cur;
            if (ok) store_out(G->out[M - 2], at, cur, o32);
#pragma unroll
            for (int t = NS - 2; t >= 0; --t) {
                if (t <= M - 2) {
                    cur = (int64_t)((uint64_t)dl[t][v] - (uint64_t)cur) >> l;  // slot t-1
                    if (ok) store_out(G->out[t == 0 ? M - 1 : t - 1], at, cur, o32);
                }
            }
            // cur is the output of slot M-1; delta_{M-1} = d_{M-1} + 2^l d_{M-2}
            if (skip < 0 && ok) {
                int64_t dr_slot = 0;
#pragma unroll
                for (int t = 0; t < NS; ++t)
                    if (t == M - 1) dr_slot = dl[t][v];
                if ((uint64_t)dr_slot != (uint64_t)cur + ((uint64_t)d_prev << l))
                    flag |= kFlagMismatch;
            }
        }
    } else if (mode == kChecksum) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (loc[v] >= lim) continue;
            uint64_t e = 0, sum = 0;
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t == M) e = (uint64_t)dl[t][v];
#pragma unroll
            for (int t = 0; t < NS - 1; ++t)
                if (t < M && t != skip) {
                    sum += (uint64_t)dl[t][v];
                    store_out(G->out[t], base + loc[v], dl[t][v], o32);
                }
            if (skip >= 0)
                store_out(G->out[skip], base + loc[v], (int64_t)(e - sum), o32);
            else if (e != sum)
                flag |= kFlagMismatch;
        }
    } else {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (t >= M || t == skip) continue;
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (loc[v] < lim) store_out(G->out[t], base + loc[v], dl[t][v], o32);
        }
    }
}

__device__ __forceinline__ bool slot_live(int skip, int t, int nslots)
{
    return t < nslots && t != skip;
}

// Byte transpose: w[a] = byte a of v[0], v[1], v[2], v[3] (in that order).
__device__ __forceinline__ void transpose4(const uint32_t *v, uint32_t *w)
{
    const uint32_t t0 = __builtin_amdgcn_perm(v[1], v[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(v[1], v[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(v[3], v[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(v[3], v[2], 0x07030602u);
    w[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    w[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    w[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    w[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Balanced digits by one add: with C = 128 (256^L - 1) / 255, u = x + C has
// ordinary base-256 digits u_a in [0, 255] exactly when x has L balanced
// digits d_a in [-128, 127], and d_a = u_a - 128, whose two's-complement
// byte is u_a ^ 0x80.
template <int L>
__device__ __forceinline__ constexpr uint64_t digit_offset()
{
    return L >= 8 ? 0x8080808080808080ull : (0x8080808080808080ull >> (64 - 8 * L));
}

// The digit bytes of a split word: the FS low bytes of a (the low field plus
// its digit offset) and then the FS low bytes of b (the high field), as one
// little-endian 64-bit value.
template <int FS>
__device__ __forceinline__ uint64_t pack_fields(uint32_t a, uint32_t b)
{
    if constexpr (FS == 1) {
        return __builtin_amdgcn_perm(b, a, 0x0c0c0400u);
    } else if constexpr (FS == 2) {
        return __builtin_amdgcn_perm(b, a, 0x05040100u);
    } else if constexpr (FS == 3) {
        return (uint64_t)__builtin_amdgcn_perm(b, a, 0x04020100u) |
               ((uint64_t)__builtin_amdgcn_perm(b, b, 0x0c0c0605u) << 32);
    } else {
        return (uint64_t)a | ((uint64_t)b << 32);
    }
}

// Stage 4 consecutive positions p..p+3 of every data word into the LA digit
// planes at ring offset `off`. Entanglement happens here, on load.
// Digit planes in LDS: plane (stream) pl occupies LAP * ring bytes; the 16
// positions starting at ring offset 16k keep their LA digit vectors (16 bytes
// each) together at pl * LAP * ring + k * 16 * LAP. LAP is LA rounded up to an
// odd count, so that the 16 lanes of an A-fragment read (16 consecutive k)
// hit 16 disjoint groups of 4 LDS banks, and each digit is an immediate
// offset 16a from one address.
template <int LA>
__device__ __forceinline__ constexpr int lap() { return LA | 1; }

__device__ __forceinline__ int plane_off(int o, int lapv) { return (o >> 4) * 16 * lapv + (o & 15); }

// Raw int32 inputs of 4 consecutive positions of the DM data streams (slot
// order), in flight between their (prefetched) global loads and their
// conversion into digit planes.
template <int DM>
struct Raw4 {
    int32_t cv[DM][4];
};

template <int DM>
__device__ __forceinline__ void load4(const GroupDev *G, int64_t p, int64_t n, Raw4<DM> &raw)
{
    if (p >= 0 && p + 4 <= n) {
#pragma unroll
        for (int m = 0; m < DM; ++m) {
            const v4i v = load_in4(G->c[m] + p);
            raw.cv[m][0] = v.x; raw.cv[m][1] = v.y; raw.cv[m][2] = v.z; raw.cv[m][3] = v.w;
        }
        return;
    }
    // Edges of the stream: zeros outside [0, n), or, for a circular
    // convolution, the window wrapped modulo n (one division per call).
    int64_t idx[4];
    bool ok[4];
    if (G->kind == kConvCircular) {
        int64_t i = p % n;
        i = i < 0 ? i + n : i;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            idx[q] = i;
            ok[q] = true;
            i = i + 1 == n ? 0 : i + 1;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            idx[q] = p + q;
            ok[q] = p + q >= 0 && p + q < n;
        }
    }
#pragma unroll
    for (int m = 0; m < DM; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) raw.cv[m][q] = ok[q] ? load_in1(G->c[m] + idx[q]) : 0;
}

// Converts raw inputs of 4 positions into the LA digit planes (one per slot,
// NP slots) at ring offset `off`: entanglement (or the checksum sum) happens
// here. Slot t entangles with slot t - 1, slot 0 with slot DM - 1.
//
// FS > 0: every word x is split at bit l into the balanced low field
// lo = x - 2^l floor(x / 2^l + 1/2) and hi = (x - lo) / 2^l (x = lo + 2^l hi),
// and each field is cut into FS digits: planes 0 .. FS-1 hold lo's digits,
// planes FS .. 2 FS - 1 hi's. Computed from x alone, like any digit split.
template <int LA, int DM, int NP, int MODE, int FS = 0>
__device__ __forceinline__ void store4(const Raw4<DM> &raw, int l, unsigned char *planes, int ring,
                                       int off, Bounds &bd)
{
    static_assert(FS == 0 || (2 * FS == LA && FS <= 4), "field digits");
    constexpr uint64_t C = digit_offset<LA>();
    constexpr int LAP = lap<LA>();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int m = 0; m + 1 < DM; m += 2) bd.add2(raw.cv[m][q], raw.cv[m + 1][q]);
        if (DM & 1) bd.add(raw.cv[DM - 1][q]);
    }
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
        uint32_t lo[4], hi[4];
        int32_t fields[4][2];  // split words: (lo, hi) of every position (FS > 0 only)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t x = 0;
            if (MODE == kChecksum && pl == DM) {
                // the sum of DM b-bit samples needs up to b + 3 bits: 64-bit adds
                int64_t sum = 0;
#pragma unroll
                for (int m = 0; m < DM; ++m) sum += raw.cv[m][q];
                x = sum;
                if constexpr (FS > 0) {
                    fields[q][0] = __builtin_amdgcn_sbfe((int32_t)sum, 0, l);
                    fields[q][1] = (int32_t)((sum - fields[q][0]) >> l);
                }
            } else if constexpr (FS > 0) {
                // The fields of x = c + 2^l c' (l <= 31; c' = 0 on raw
                // words) without forming it: x's low l bits are c's, so
                // lo = c's low l bits sign-extended, hi = c' + (c - lo) / 2^l
                // (an exact shift). Unsigned wrap keeps inputs outside the
                // declared range (flagged) well defined.
                const int32_t c = raw.cv[pl % DM][q];
                const int32_t cp = MODE == kEntangled ? raw.cv[(pl + DM - 1) % DM][q] : 0;
                fields[q][0] = __builtin_amdgcn_sbfe(c, 0, l);
                fields[q][1] = (int32_t)((uint32_t)cp +
                                         (uint32_t)((int32_t)((uint32_t)c - (uint32_t)fields[q][0]) >> l));
            } else if (MODE == kEntangled) {
                x = ent(raw.cv[pl % DM][q], raw.cv[(pl + DM - 1) % DM][q], l);
            } else {
                x = raw.cv[pl % DM][q];
            }
            // (x has LA digits whenever the inputs lie in the declared range,
            // which the plan sized LA for and the kernel verifies.)
            uint64_t u;
            if constexpr (FS > 0) {
                constexpr uint32_t CF = (uint32_t)digit_offset<FS>();
                u = pack_fields<FS>((uint32_t)fields[q][0] + CF, (uint32_t)fields[q][1] + CF);
            } else {
                u = (uint64_t)x + C;
            }
            lo[q] = (uint32_t)u;
            hi[q] = (uint32_t)(u >> 32);
        }
        uint32_t w[8];
        transpose4(lo, w);
        if (LA > 4) transpose4(hi, w + 4);
        unsigned char *dst = planes + (size_t)pl * LAP * ring + plane_off(off, LAP);
#pragma unroll
        for (int a = 0; a < LA; ++a) *reinterpret_cast<uint32_t *>(dst + 16 * a) = w[a] ^ 0x80808080u;
    }
}

// ----------------------------------------------------- convolution kernel

// The LDS words of one tap-operand fragment: 4 aligned words, or the 5
// aligned words that cover 16 bytes at any byte shift.
template <int TC>
struct TapWords {
    static constexpr int n = TC == 4 ? 4 : 5;
    uint32_t w[n];
};

// Digit pairs of the convolution's products. The accumulator of data digit a
// and tap digit b is acc_of(a) + b: weight a + b, or, for words split into
// fields of FS digits, the high field's weights after the SL = FS + LB - 1 of
// the low field. Without a split a pair of weight 256^8 or more is a multiple
// of 2^64 and does not run; with one every pair runs (the high field's weight
// 2^l 256^(a + b) depends on the group's l). Pairs run b-major, a-minor:
// pair_first says which one writes its accumulator first.
template <int FS, int LB>
__device__ __forceinline__ constexpr int acc_of(int a)
{
    return FS && a >= FS ? a + LB - 1 : a;
}
template <int FS>
__device__ __forceinline__ constexpr bool pair_runs(int a, int b)
{
    return FS ? true : a + b < 8;
}
template <int LA, int FS>
__device__ __forceinline__ constexpr bool pair_first(int a, int b)
{
    return b == 0 || a == LA - 1 || (FS && a == FS - 1);
}

// One variant per kernel class (0 entangled, 1 plain, 2 checksum) and slot
// count NS, so that the mode, M and the slot loop are compile-time: the
// descriptor's mode and M must match (the planner picks the variant).
//
// GW waves share one staging ring. GW = 4: the block's ring covers 1024
// outputs per step (each wave a 256-output tile of it); every wave stages a
// quarter of the new positions, so two block barriers per step order the
// staging against the reads. GW = 1: each wave owns a ring and a sub-strip
// of steps x 256 outputs (the block's strip split in four) and stages its
// own positions; a wave's LDS accesses take effect in program order, so the
// step loop has no barrier at all, at the price of a window of kp extra
// positions per wave instead of per block.
// TC: copies of each tap-digit plane (4, or 1 with GW = 4, below).
// FS: digits per field of words split at bit l (0: not split; LA = 2 FS).
// conv_item runs one work item (a strip of one group); k_conv_fused is one
// launch over a bucket of items of this variant.
template <int LA, int LB, int NS, int KCLASS, int GW, int SP, int TC, int FS = 0>
__device__ __forceinline__ void conv_item(const GroupDev *__restrict__ groups, const Item it,
                                          uint32_t *flags)
{
    constexpr int mode = KCLASS == 0 ? kEntangled : (KCLASS == 2 ? kChecksum : kPlain);
    constexpr int M = KCLASS == 2 ? NS - 1 : NS;  // data streams
    constexpr int nplanes = NS;
    static_assert(M >= 1 && M <= kFusedMaxM, "slot count");
    static_assert(GW == 1 || GW == 4, "waves per ring");
    static_assert(SP == 0 || (SP == 1 && LB >= 2), "sparse top tap digit");
    static_assert(TC == 4 || (TC == 1 && GW == 4), "tap-plane copies");
    static_assert(FS == 0 || (2 * FS == LA && SP == 0), "split words");
    constexpr int LBM = LB - SP;     // tap digit planes of the main pass
    constexpr int SPAN = 256 * GW;   // positions a ring advances per step
    constexpr int GT = 64 * GW;      // threads staging one ring
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const GroupDev *G = groups + it.g;
    const int skip = G->skip, l = G->l;
    const int nch = G->nch, kp = G->kp;
    const int ring = SPAN + kp;  // window of one step, a multiple of 16
    const int steps = G->steps, acc16 = G->acc16, use_dma = G->dma;
    const int64_t n = G->n, K = G->K, n_out = G->n_out;
    const int32_t *__restrict__ g = G->operand;
    const int tid = item_tid(), lane = tid & 63, wave = tid >> 6;
    const int grp = wave / GW, wg = wave % GW, gt = tid % GT;  // ring, wave and thread in it
    uint32_t flag = 0;
    Bounds bd;

    // LDS: tap-digit planes | data digit-plane rings | raw inputs.
    //
    // The Toeplitz operand B[s][j] = g[j + kp - s] is not stored expanded
    // (each tap would appear 16 times): with the reversed taps
    // Q[v] = g[kp + 15 - v], lane (j, h) of chunk c needs the 16 bytes
    // Q[64c + 16h + 15 - j ...], consecutive but at a byte alignment set by
    // j. With TC = 4 copies per digit plane, copy r shifted by (4 - r) mod 4
    // bytes, the lane reads its fragment as 4 dword-aligned words from the
    // copy matching its alignment; with one copy it reads the 5 aligned
    // words that cover the fragment and shifts them into place.
    const int tpb = (int)conv_tap_plane_bytes(nch);
    unsigned char *taps = smem;
    // Bit c of tmask: chunk c's top tap-digit plane has a nonzero digit
    // (sparse-top variants; chunks from 64 on always run it).
    uint32_t *tmask = reinterpret_cast<uint32_t *>(smem + (size_t)TC * LB * tpb);
    const size_t ring0 = (size_t)TC * LB * tpb + 16;
    unsigned char *planes = smem + ring0 + (size_t)grp * nplanes * lap<LA>() * ring;
    if (SP) {
        if (tid < 2) tmask[tid] = 0;
        __syncthreads();
    }
    {
        constexpr uint64_t CB = digit_offset<LB>();
        const int vlen = 64 * nch + 16;
        const bool xcorr = G->kind == kConvXcorr;  // cross-correlation: the taps reversed
        for (int v = tid; v < vlen; v += kBlock) {
            const int64_t idx = (int64_t)kp + 15 - v;
            const int32_t gv = (idx >= 0 && idx < K) ? g[xcorr ? K - 1 - idx : idx] : 0;
            bd.add(gv);
            const uint64_t u = (uint64_t)(int64_t)gv + CB;
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const unsigned char d = (unsigned char)((u >> (8 * b)) & 0xffu) ^ 0x80u;
                if constexpr (TC == 4) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) taps[(b * 4 + r) * tpb + ((4 - r) & 3) + v] = d;
                } else {
                    taps[b * tpb + v] = d;
                }
                if (SP && b == LB - 1 && d != 0) {
                    // the chunks whose fragments read Q[v]: 64c <= v <= 64c + 78
                    for (int c = v >> 6; c >= 0 && 64 * c + 78 >= v; --c)
                        if (c < 64) atomicOr(&tmask[c >> 5], 1u << (c & 31));
                }
            }
        }
    }
    // This lane's fragment of plane b, chunk c: at tap_lane + TC b tpb + 64 c,
    // 4 aligned words (TC = 4), or 16 bytes at byte shift tsh from an aligned
    // word (TC = 1). The words are loaded as they lie and shifted into place
    // only when the fragment is used, so that a load in flight is not waited
    // for early.
    const int tj = lane & 15, th = lane >> 4;
    const int tr = (15 - tj) & 3;
    const int tap_lane = TC == 4 ? tr * tpb + ((4 - tr) & 3) + 16 * th + 15 - tj
                                 : (16 * th + 15 - tj) & ~3;
    const uint32_t tsh = (uint32_t)(15 - tj) & 3u;
    auto tap_load = [&](int b, int c, TapWords<TC> &t) {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(taps + tap_lane + TC * b * tpb + 64 * c);
#pragma unroll
        for (int i = 0; i < TapWords<TC>::n; ++i) t.w[i] = q[i];
    };
    auto tap_frag = [&](const TapWords<TC> &t) -> v4i {
        if constexpr (TC == 4) {
            return v4i{(int)t.w[0], (int)t.w[1], (int)t.w[2], (int)t.w[3]};
        } else {
            return v4i{(int)__builtin_amdgcn_alignbyte(t.w[1], t.w[0], tsh),
                       (int)__builtin_amdgcn_alignbyte(t.w[2], t.w[1], tsh),
                       (int)__builtin_amdgcn_alignbyte(t.w[3], t.w[2], tsh),
                       (int)__builtin_amdgcn_alignbyte(t.w[4], t.w[3], tsh)};
        }
    };

    // The digit planes are rings of `ring` bytes (the window SPAN + kp, a
    // multiple of 16, so no 16-byte access wraps): ring offset 0 is position
    // T0 - kp. The first step stages the whole window, every later step only
    // its SPAN new positions, at ring offsets that advance by SPAN per step.
    const int64_t T0 = (int64_t)it.strip * steps * kConvTile + (int64_t)grp * steps * SPAN;
    const int64_t base = T0 - kp;
    {
        Raw4<M> raw;
        for (int gi = gt; gi < (ring >> 2); gi += GT) {
            load4<M>(G, base + 4 * gi, n, raw);
            store4<LA, M, nplanes, mode, FS>(raw, l, planes, ring, 4 * gi, bd);
        }
    }
    __syncthreads();  // tap planes (and the first windows) complete
    uint64_t topmask = 0;
    if (SP)
        topmask = ((uint64_t)__builtin_amdgcn_readfirstlane(tmask[1]) << 32) |
                  __builtin_amdgcn_readfirstlane(tmask[0]);
    // The raw int32 inputs of the next step travel HBM -> LDS by direct
    // loads (global_load_lds_dwordx4, no registers held) while this step
    // computes; the lane of staging thread j fetches positions 4j .. +3 of
    // every stream, exactly the positions thread j converts at the step
    // boundary, so only the wave's own wait is needed before converting.
    // Lanes whose 4 positions are not all inside [0, n) load nothing; their
    // positions are read with bounds checks at conversion.
    unsigned char *rawb = smem + ring0 + (size_t)(4 / GW) * nplanes * lap<LA>() * ring;
    auto dma = [&](int64_t Tq) {
        const int64_t p = Tq + 4 * gt;
        if (use_dma && p + 4 <= n) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(G->c[m] + p),
                        (__attribute__((address_space(3))) void *)(rawb + m * 4096 + wave * 1024),
                        16, 0, 0);
        }
    };
    if (steps > 1 && T0 + SPAN < n_out) dma(T0 + SPAN);

    int loc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) loc[v] = 16 * (4 * (lane >> 4) + v) + (lane & 15);
    // Ring offsets: this lane's A-fragment row (16 positions) of the current
    // step, and this thread's 4 staged positions of the next step.
    int aoff = 256 * wg + 16 * (lane & 15) + 16 * (lane >> 4);
    int soff = 4 * gt;

    for (int step = 0; step < steps; ++step) {
        const int64_t T = T0 + (int64_t)step * SPAN;
        if (T >= n_out) break;
        if (GW > 1 && step > 0) __syncthreads();  // digit planes of this step complete

        // Without the LDS prefetch, block-ring variants load the next
        // step's raw inputs into registers here, so that they arrive while
        // this step computes (per-wave ring variants, which keep fewer
        // registers, load them at the step boundary).
        const int64_t Tn = T + SPAN;
        const bool more = step + 1 < steps && Tn < n_out;
        Raw4<M> pre;
        if (GW > 1 && !use_dma && more) load4<M>(G, Tn + 4 * gt, n, pre);

        // Each wave: its 16x16 output tile, for every live slot.
        const int64_t P0 = T + 256 * wg;
        int64_t dl[NS][4];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (t == skip) {
                // never read; a copy of a defined value keeps the compiler
                // from carrying undefined registers around the step loop
#pragma unroll
                for (int v = 0; v < 4; ++v) dl[t][v] = t > 0 ? dl[t > 0 ? t - 1 : 0][v] : 0;
                continue;
            }
            const unsigned char *pbase = planes + (size_t)t * lap<LA>() * ring;
            // One accumulator per digit weight s = a + b: the matrix core
            // sums the digit pairs of equal weight. A pair with a + b >= 8 is
            // a multiple of 2^64 and is skipped. Chunk 0 (there is always
            // one) starts every weight from zero. Split words: weights
            // 256^s of the low field in acc[0 .. SL), 2^l 256^s of the high
            // field in acc[SL ..); every pair runs (l is not known here).
            constexpr int SL = FS + LB - 1;
            constexpr int S = FS ? 2 * SL : ((LA + LB - 1) < 8 ? (LA + LB - 1) : 8);
            v4i acc[S];
            // Byte offset of this lane's A row in the slot's digit planes:
            // ring offsets here are multiples of 16, where plane_off(o) is
            // o * LAP, so the offset advances by 64 LAP a chunk and wraps
            // by one unsigned min (offset - ring LAP wraps above the offset
            // exactly when the offset is below ring LAP).
            uint32_t ob = (uint32_t)aoff * lap<LA>();
            const uint32_t ringb = (uint32_t)ring * lap<LA>();
            using TW = TapWords<TC>;
            auto load = [&](int c, TW(&bf)[LBM], v4i(&af)[LA]) {
                const unsigned char *pa = pbase + ob;
                ob += 64 * lap<LA>();
                ob = min(ob, ob - ringb);
#pragma unroll
                for (int b = 0; b < LBM; ++b) tap_load(b, c, bf[b]);
#pragma unroll
                for (int a = 0; a < LA; ++a) af[a] = *reinterpret_cast<const v4i *>(pa + 16 * a);
            };
            auto mma = [&](const TW(&bw)[LBM], const v4i(&af)[LA]) {
#pragma unroll
                for (int b = 0; b < LBM; ++b) {
                    const v4i bf = tap_frag(bw[b]);
#pragma unroll
                    for (int a = 0; a < LA; ++a)
                        if (pair_runs<FS>(a, b))
                            acc[acc_of<FS, LB>(a) + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                af[a], bf, acc[acc_of<FS, LB>(a) + b], 0, 0, 0);
                }
            };
            // chunk 0 starts every weight the main pass reaches (its first pair
            // writes it with a zero accumulator); a weight only the sparse top
            // plane reaches starts at zero
            auto mma_first = [&](const TW(&bw)[LBM], const v4i(&af)[LA]) {
                if (SP && LA + LB - 2 < 8) acc[LA + LB - 2] = v4i{0, 0, 0, 0};
#pragma unroll
                for (int b = 0; b < LBM; ++b) {
                    const v4i bf = tap_frag(bw[b]);
#pragma unroll
                    for (int a = 0; a < LA; ++a)
                        if (pair_runs<FS>(a, b))
                            acc[acc_of<FS, LB>(a) + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                af[a], bf,
                                pair_first<LA, FS>(a, b) ? v4i{0, 0, 0, 0}
                                                         : acc[acc_of<FS, LB>(a) + b],
                                0, 0, 0);
                }
            };
            if constexpr (GW == 1) {
                // Per-wave rings serve short kernels (few chunks): one
                // fragment buffer, fewer registers, more waves per SIMD.
                {
                    TW bf[LBM];
                    v4i af[LA];
                    load(0, bf, af);
                    mma_first(bf, af);
                }
                for (int c = 1; c < nch; ++c) {
                    TW bf[LBM];
                    v4i af[LA];
                    load(c, bf, af);
                    mma(bf, af);
                }
            } else {
                // Block rings serve long kernels (many chunks). Two fragment
                // buffers: the loads of chunk c + 1 are in flight while the
                // matrix cores work on chunk c. Each half step first waits for
                // every LDS load (only the current buffer's are in flight),
                // then issues the next chunk's loads, then the current chunk's
                // products; the scheduling barriers keep that order.
                auto half = [&](int cn, bool more, TW(&bfn)[LBM], v4i(&afn)[LA],
                                const TW(&bfc)[LBM], const v4i(&afc)[LA]) {
                    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) load(cn, bfn, afn);
                    __builtin_amdgcn_sched_barrier(0);
                    mma(bfc, afc);
                };
                TW bf0[LBM], bf1[LBM];
                v4i af0[LA], af1[LA];
                load(0, bf0, af0);
                __builtin_amdgcn_s_waitcnt(0xc07f);
                __builtin_amdgcn_sched_barrier(0);
                if (nch > 1) load(1, bf1, af1);
                __builtin_amdgcn_sched_barrier(0);
                mma_first(bf0, af0);
                for (int c = 1; c < nch; c += 2) {
                    half(c + 1, c + 1 < nch, bf0, af0, bf1, af1);  // products of chunk c
                    if (c + 1 >= nch) break;
                    half(c + 2, c + 2 < nch, bf1, af1, bf0, af0);  // products of chunk c + 1
                }
            }
            if constexpr (SP) {
                // the top tap-digit plane, only for the chunks whose taps need it
                auto top = [&](int c) {
                    int ot = aoff + 64 * c;
                    ot = ot >= ring ? ot - ring : ot;
                    const unsigned char *pa = pbase + (uint32_t)ot * lap<LA>();
                    TapWords<TC> tw;
                    tap_load(LB - 1, c, tw);
                    const v4i bt = tap_frag(tw);
                    v4i af[LA];
#pragma unroll
                    for (int a = 0; a < LA; ++a) af[a] = *reinterpret_cast<const v4i *>(pa + 16 * a);
#pragma unroll
                    for (int a = 0; a < LA; ++a)
                        if (a + LB - 1 < 8)
                            acc[a + LB - 1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                af[a], bt, acc[a + LB - 1], 0, 0, 0);
                };
                uint64_t m = nch >= 64 ? topmask : topmask & ((1ull << nch) - 1);
                for (; m; m &= m - 1) top(__builtin_ctzll(m));
                for (int c = 64; c < nch; ++c) top(c);
            }
            // y = sum_s 256^s acc_s (mod 2^64). When the plan has shown every
            // acc_s + 256 acc_{s+1} fits in int32 (acc16), neighbouring digit
            // sums are merged in 32 bits first and the 64-bit Horner steps
            // over 16-bit shifts.
            constexpr int H = (S + 1) / 2;
            if constexpr (FS > 0) {
                // y = lo + 2^l hi, each field's sum sum_s 256^s acc_s in 32
                // bits when the plan has shown it fits (acc16), else in 64
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    uint64_t ylo, yhi;
                    if (acc16) {
                        uint32_t zl = (uint32_t)acc[SL - 1][v], zh = (uint32_t)acc[S - 1][v];
#pragma unroll
                        for (int k = SL - 2; k >= 0; --k) {
                            zl = (zl << 8) + (uint32_t)acc[k][v];
                            zh = (zh << 8) + (uint32_t)acc[SL + k][v];
                        }
                        ylo = (uint64_t)(int64_t)(int32_t)zl;
                        yhi = (uint64_t)(int64_t)(int32_t)zh;
                    } else {
                        ylo = (uint64_t)(int64_t)acc[SL - 1][v];
                        yhi = (uint64_t)(int64_t)acc[S - 1][v];
#pragma unroll
                        for (int k = SL - 2; k >= 0; --k) {
                            ylo = (ylo << 8) + (uint64_t)(int64_t)acc[k][v];
                            yhi = (yhi << 8) + (uint64_t)(int64_t)acc[SL + k][v];
                        }
                    }
                    dl[t][v] = (int64_t)(ylo + (yhi << l));
                }
            } else if (acc16) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int32_t z[H];
#pragma unroll
                    for (int k = 0; k < H; ++k)
                        z[k] = (int32_t)((uint32_t)acc[2 * k][v] +
                                         (2 * k + 1 < S ? (uint32_t)acc[(2 * k + 1) % S][v] << 8
                                                        : 0u));
                    uint64_t y = (uint64_t)(int64_t)z[H - 1];
#pragma unroll
                    for (int k = H - 2; k >= 0; --k) y = (y << 16) + (uint64_t)(int64_t)z[k];
                    dl[t][v] = (int64_t)y;
                }
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    uint64_t y = (uint64_t)(int64_t)acc[S - 1][v];
#pragma unroll
                    for (int s = S - 2; s >= 0; --s) y = (y << 8) + (uint64_t)(int64_t)acc[s][v];
                    dl[t][v] = (int64_t)y;
                }
            }
        }

        // Raw inputs of the next step are fetched before this step's outputs
        // are stored, so that waiting for the direct loads does not also wait
        // for those stores.
        if (more) {
            Raw4<M> raw = pre;
            const int64_t p = Tn + 4 * gt;
            if (GW > 1 && !use_dma) {
                // loaded at the top of the step
            } else if (use_dma && p + 4 <= n) {
                __builtin_amdgcn_s_waitcnt(0);  // this wave's direct loads have landed
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int4 v = *reinterpret_cast<const int4 *>(rawb + m * 4096 + 16 * tid);
                    raw.cv[m][0] = v.x; raw.cv[m][1] = v.y; raw.cv[m][2] = v.z; raw.cv[m][3] = v.w;
                }
            } else {
                load4<M>(G, p, n, raw);
            }
            epilogue<NS, 4>(G, mode, M, skip, l, P0, n_out - P0, loc, dl, flag);
            if (GW > 1) __syncthreads();  // every wave is done with the ring slots reused here
            store4<LA, M, nplanes, mode, FS>(raw, l, planes, ring, soff, bd);
            if (step + 2 < steps && Tn + SPAN < n_out) dma(Tn + SPAN);
        } else {
            epilogue<NS, 4>(G, mode, M, skip, l, P0, n_out - P0, loc, dl, flag);
        }
        aoff += SPAN;
        aoff = aoff >= ring ? aoff - ring : aoff;
        soff += SPAN;
        soff = soff >= ring ? soff - ring : soff;
    }
    if (bd.lo < G->in_lo || bd.hi > G->in_hi) flag |= kFlagInputRange;
    if (flag) atomicOr(flags, flag);
}

template <int LA, int LB, int NS, int KCLASS, int GW, int SP, int TC, int FS = 0>
__global__ __launch_bounds__(kBlock) void k_conv_fused(const GroupDev *__restrict__ groups,
                                                       const Item *__restrict__ items,
                                                       uint32_t nitems, uint32_t *flags)
{
    const uint32_t ii = item_index(nitems);
    if (ii >= nitems) return;
    conv_item<LA, LB, NS, KCLASS, GW, SP, TC, FS>(groups, items[ii], flags);
}

// ------------------------------------------------ element-wise operations

// V consecutive int32 values (V = 2: one 8-byte load, V = 4: one 16-byte
// load, V = 8: two).
template <int V, typename T>
__device__ __forceinline__ void load_vec(const int32_t *src, T (&x)[V])
{
    if constexpr (V == 8) {
        const int4 w = *reinterpret_cast<const int4 *>(src);
        const int4 u = *reinterpret_cast<const int4 *>(src + 4);
        x[0] = w.x; x[1] = w.y; x[2] = w.z; x[3] = w.w;
        x[4] = u.x; x[5] = u.y; x[6] = u.z; x[7] = u.w;
    } else if constexpr (V == 4) {
        const int4 w = *reinterpret_cast<const int4 *>(src);
        x[0] = w.x; x[1] = w.y; x[2] = w.z; x[3] = w.w;
    } else {
        const int2 w = *reinterpret_cast<const int2 *>(src);
        x[0] = w.x; x[1] = w.y;
    }
}

// Recovery of V consecutive positions per lane with the results left in
// place: on return dl[t][v] holds the recovered output of slot t (entangled:
// stream (r + 1 + t) mod M; otherwise stream t), for t < M. Same arithmetic
// as epilogue(); with stream r computed, the redundant slot is checked.
template <int NS, int V>
__device__ __forceinline__ void recover_inplace(int mode, int M, int skip, int l,
                                                int64_t (&dl)[NS][V], uint32_t &flag)
{
    if (mode == kEntangled) {
        const int s = 64 - (M - 1) * l;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            uint64_t acc = 0;
#pragma unroll
            for (int t = 0; t < NS - 1; ++t)
                if (t < M - 1) {
                    const uint64_t x = (uint64_t)dl[t][v];
                    acc = (acc << l) + (((M + t) & 1) ? (uint64_t)0 - x : x);
                }
            int64_t cur = ((int64_t)(acc << s)) >> s;  // d of slot M-2
            const int64_t d_prev = cur;
#pragma unroll
            for (int t = NS - 2; t >= 0; --t)
                if (t <= M - 2) {
                    const int64_t delta = dl[t][v];
                    dl[t][v] = cur;                                              // d of slot t
                    cur = (int64_t)((uint64_t)delta - (uint64_t)cur) >> l;      // d of slot t-1
                }
            // cur is d_r (slot M-1)
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t == M - 1) {
                    if (skip < 0 && (uint64_t)dl[t][v] != (uint64_t)cur + ((uint64_t)d_prev << l))
                        flag |= kFlagMismatch;
                    dl[t][v] = cur;
                }
        }
    } else if (mode == kChecksum) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            uint64_t e = 0, sum = 0;
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t == M) e = (uint64_t)dl[t][v];
#pragma unroll
            for (int t = 0; t < NS - 1; ++t)
                if (t < M && t != skip) sum += (uint64_t)dl[t][v];
            if (skip >= 0) {
#pragma unroll
                for (int t = 0; t < NS - 1; ++t)
                    if (t == skip) dl[t][v] = (int64_t)(e - sum);
            } else if (e != sum) {
                flag |= kFlagMismatch;
            }
        }
    }
}

// Permutation groups first have their streams interleaved into rows of RW
// int32 (RW = 4 for up to 4 slots, else 8; unused entries zero) in the plan's
// workspace: a row holds every stream's sample of one position, so that the
// gather at pi[i] reads one 16- or 32-byte row instead of M scattered words.
// A layout change only; no arithmetic. 4 positions per lane per step.
// steps: 1024-position steps per work item (strip it.strip of that length).
template <int RW>
__device__ __forceinline__ void interleave_item(const GroupDev *__restrict__ groups, const Item it,
                                                int steps)
{
    const GroupDev *G = groups + it.g;
    const int M = G->M;
    const int64_t n = G->n;
    const int tid = item_tid();
    int32_t *__restrict__ rows = G->rows;
    const int64_t strip0 = (int64_t)it.strip * steps * kBlock * 4;
    for (int q = 0; q < steps; ++q) {
        const int64_t p = strip0 + (int64_t)q * kBlock * 4 + 4 * tid;
        if (p >= n) break;
        const bool full = p + 4 <= n;
        int32_t x[RW][4];
#pragma unroll
        for (int t = 0; t < RW; ++t) {
#pragma unroll
            for (int v = 0; v < 4; ++v) x[t][v] = 0;
            if (t < M) {
                if (full) {
                    const v4i w = load_in4(G->c[t] + p);
                    x[t][0] = w.x; x[t][1] = w.y; x[t][2] = w.z; x[t][3] = w.w;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (p + v < n) x[t][v] = load_in1(G->c[t] + p + v);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (p + v >= n) continue;
#pragma unroll
            for (int h = 0; h < RW; h += 4)
                *reinterpret_cast<v4i *>(rows + (p + v) * RW + h) =
                    v4i{x[h][v], x[h + 1][v], x[h + 2][v], x[h + 3][v]};
        }
    }
}

template <int RW>
__global__ __launch_bounds__(kBlock) void k_interleave(const GroupDev *__restrict__ groups,
                                                       const Item *__restrict__ items,
                                                       uint32_t nitems)
{
    const uint32_t ii = blockIdx.x;
    if (ii >= nitems) return;
    const Item it = items[ii];
    interleave_item<RW>(groups, it, groups[it.g].steps);
}

// Scale, add, permutation and inner product: V consecutive positions per
// lane per step (8- or 16-byte loads, 16-byte stores), all M streams of the group at
// once (entangle -> op -> recover in registers). The descriptor holds the
// streams in slot order, so the previous stream of slot t >= 1 is slot t - 1
// (of slot 0: slot M - 1) and no register is selected at run time. Inner products accumulate per slot into the group's
// accumulators; k_inner_finalize recovers them.
//
// One variant per operation, kernel class (0 entangled, 1 plain, 2 checksum)
// and slot count NS: operation, mode, M and the slot loops are compile-time.
//
// Items are taken in plain block order (no per-XCD runs): neighbouring
// blocks then work on the same group at the same time, so a permutation's
// random gathers fall into a working set the memory-side cache holds.
// VX: a multiple of stream_positions(NS) per lane (stream_positions_of: 2
// for gathers and inner products, for more loads in flight).
template <int OP, int KCLASS, int NS, int VX = 1>
__device__ __forceinline__ void stream_item(const GroupDev *__restrict__ groups, const Item it,
                                            uint32_t *flags)
{
    constexpr int V = stream_positions(NS) * VX;
    constexpr int op = OP;
    constexpr int mode = KCLASS == 0 ? kEntangled : (KCLASS == 2 ? kChecksum : kPlain);
    constexpr int M = KCLASS == 2 ? NS - 1 : NS;
    constexpr int nslots = NS;
    static_assert(V == 2 || V == 4 || V == 8, "2, 4 or 8 positions per lane");
    const GroupDev *G = groups + it.g;
    const int tid = item_tid();
    const int skip = G->skip, l = G->l;
    const int steps = G->steps;
    // the outer product iterates over its n K outputs: output o takes input
    // o / K and operand value o mod K
    const int64_t n = op == NE_OP_OUTER ? G->n_out : G->n, sv = G->scalar;
    const int64_t K = G->K;
    const int32_t *__restrict__ opd = G->operand;
    uint32_t flag = 0;
    Bounds bd;
    uint64_t iacc[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) iacc[t] = 0;
    const int64_t strip0 = (int64_t)it.strip * steps * kBlock * V;
    for (int q = 0; q < steps; ++q) {
        const int64_t pb = strip0 + (int64_t)q * kBlock * V;
        if (pb >= n) break;
        const int64_t p = pb + V * tid;
        const bool full = p + V <= n;
        int64_t src[V];
        int64_t gj[V];
#pragma unroll
        for (int v = 0; v < V; ++v) src[v] = p + v < n ? p + v : 0;
        if (op == NE_OP_OUTER) {
            // one division per lane and step; (i, j) then advance by one
            int64_t i = p / K, j = p - i * K;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                src[v] = p + v < n ? i : 0;
                gj[v] = p + v < n ? j : 0;
                if (++j == K) {
                    j = 0;
                    ++i;
                }
            }
        }
        if (op == NE_OP_PERM) {
            if (full) {
                load_vec<V>(opd + p, src);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) src[v] = p + v < n ? opd[p + v] : 0;
            }
            // an index outside [0, n) is not a permutation index: it is
            // flagged, and row 0 is read in its place (defined memory)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (src[v] < 0 || src[v] >= n) {
                    flag |= kFlagPermIndex;
                    src[v] = 0;
                }
            }
        }
        auto load = [&](const int32_t *base, int32_t (&x)[V]) {
            if (op != NE_OP_PERM && op != NE_OP_OUTER && full) {
                load_vec<V>(base + p, x);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) x[v] = p + v < n ? base[src[v]] : 0;
            }
        };
        // Inputs in slot order; prev0: the partner of slot 0 (slot M - 1).
        // csum: the checksum stream's sample, summed in 64 bits (M b-bit
        // samples need up to b + 3 bits)
        int32_t cv[NS][V], prev0[V], gv[V];
        int64_t csum[V];
#pragma unroll
        for (int v = 0; v < V; ++v) csum[v] = prev0[v] = gv[v] = 0;
#pragma unroll
        for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int v = 0; v < V; ++v) cv[t][v] = 0;
        if (op == NE_OP_PERM) {
            // one interleaved row per position (k_interleave)
            constexpr int RW = NS <= 4 ? 4 : 8;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (p + v >= n) continue;
                const int32_t *row = G->rows + src[v] * RW;
#pragma unroll
                for (int h = 0; h < RW; h += 4) {
                    const v4i w = *reinterpret_cast<const v4i *>(row + h);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (h + e < NS) cv[h + e][v] = w[e];
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t < M) load(G->c[t], cv[t]);
        }
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (t < M) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    bd.add(cv[t][v]);
                    csum[v] += cv[t][v];
                }
            }
        }
        if (mode == kEntangled) {
#pragma unroll
            for (int t = 0; t < NS; ++t)
                if (t == M - 1)
#pragma unroll
                    for (int v = 0; v < V; ++v) prev0[v] = cv[t][v];
        }
        if (op == NE_OP_ADD || op == NE_OP_SUB || op == NE_OP_MUL || op == NE_OP_INNER) {
            if (full) {
                load_vec<V>(opd + p, gv);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) gv[v] = p + v < n ? opd[p + v] : 0;
            }
#pragma unroll
            for (int v = 0; v < V; ++v) bd.add(gv[v]);
        } else if (op == NE_OP_OUTER) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                gv[v] = p + v < n ? opd[gj[v]] : 0;
                bd.add(gv[v]);
            }
        }
        int64_t dl[NS][V];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                dl[t][v] = 0;
                if (!slot_live(skip, t, nslots)) continue;
                int64_t x, gs = gv[v];
                if (mode == kEntangled) {
                    x = ent(cv[t][v], t == 0 ? prev0[v] : cv[t == 0 ? 0 : t - 1][v], l);
                    gs = ent(gv[v], gv[v], l);  // footnote 3: the added vector is entangled too
                } else if (mode == kChecksum && t == M) {
                    x = csum[v];
                    gs = (int64_t)M * gv[v];  // checksum of the M added operands
                } else {
                    x = cv[t][v];
                }
                uint64_t y;
                switch (op) {
                case NE_OP_SCALE: y = (uint64_t)x * (uint64_t)sv; break;
                case NE_OP_ADD: y = (uint64_t)x + (uint64_t)gs; break;
                case NE_OP_SUB: y = (uint64_t)x - (uint64_t)gs; break;
                case NE_OP_MUL:
                case NE_OP_OUTER: y = (uint64_t)x * (uint64_t)(int64_t)gv[v]; break;
                case NE_OP_INNER: y = (uint64_t)x * (uint64_t)(int64_t)gv[v]; break;
                default: y = (uint64_t)x; break;  // permutation: the gather above
                }
                if (op == NE_OP_INNER)
                    iacc[t] += (p + v < n) ? y : 0;
                else
                    dl[t][v] = (int64_t)y;
            }
        }
        if (op == NE_OP_INNER) continue;
        recover_inplace<NS, V>(mode, M, skip, l, dl, flag);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            if (t >= M || (mode != kEntangled && mode != kChecksum && t == skip)) continue;
            if (G->out32) {
                int32_t *o = (int32_t *)G->out[t] + p;
                if (full) {
                    if constexpr (V >= 4) {
#pragma unroll
                        for (int v = 0; v < V; v += 4)
                            *reinterpret_cast<v4i *>(o + v) =
                                v4i{(int32_t)dl[t][v], (int32_t)dl[t][v + 1], (int32_t)dl[t][v + 2],
                                    (int32_t)dl[t][v + 3]};
                    } else {
                        *reinterpret_cast<int2 *>(o) = int2{(int32_t)dl[t][0], (int32_t)dl[t][1]};
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (p + v < n) o[v] = (int32_t)dl[t][v];
                }
            } else {
                int64_t *o = G->out[t] + p;
                if (full) {
#pragma unroll
                    for (int v = 0; v < V; v += 2)
                        *reinterpret_cast<I64x2 *>(o + v) = I64x2{dl[t][v], dl[t][v + 1]};
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (p + v < n) o[v] = dl[t][v];
                }
            }
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
            if ((tid & 63) == 0) part[tid >> 6][t] = v;
        }
        __syncthreads();
        if (tid < NS && tid < nslots) {
            uint64_t s = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += part[w][tid];
            atomicAdd(reinterpret_cast<unsigned long long *>(G->acc + tid),
                      (unsigned long long)s);
        }
    }
    if (bd.lo < G->in_lo || bd.hi > G->in_hi) flag |= kFlagInputRange;
    if (flag) atomicOr(flags, flag);
}

template <int OP, int KCLASS, int NS, int VX = 1>
__global__ __launch_bounds__(kBlock) void k_stream_fused(const GroupDev *__restrict__ groups,
                                                         const Item *__restrict__ items,
                                                         uint32_t nitems, uint32_t *flags)
{
    const uint32_t ii = blockIdx.x;
    if (ii >= nitems) return;
    stream_item<OP, KCLASS, NS, VX>(groups, items[ii], flags);
}

// Recovery of one group's inner products (one output per stream) from its
// accumulated partial sums; also clears the accumulators for the next run.
// ATOMIC: read and clear each accumulator with one device-scope exchange
// (when the partial sums came from other blocks of the same launch).
template <int NS, bool ATOMIC = false>
__device__ __forceinline__ void inner_finalize_group(const GroupDev *__restrict__ G,
                                                     uint32_t *flags)
{
    uint32_t flag = 0;
    int64_t dl[NS][1];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        if constexpr (ATOMIC) {
            dl[t][0] = (int64_t)atomicExch(reinterpret_cast<unsigned long long *>(G->acc + t), 0ull);
        } else {
            dl[t][0] = (int64_t)G->acc[t];
            G->acc[t] = 0;
        }
    }
    const int loc[1] = {0};
    epilogue<NS, 1>(G, G->mode, G->M, G->skip, G->l, 0, 1, loc, dl, flag);
    if (flag) atomicOr(flags, flag);
}

// Recovery of inner products after all partial sums have landed (a launch
// of its own, after the element-wise launches).
template <int NS>
__global__ __launch_bounds__(64) void k_inner_finalize(const GroupDev *__restrict__ groups,
                                                       const uint32_t *__restrict__ gidx,
                                                       uint32_t count, uint32_t *flags)
{
    const uint32_t i = blockIdx.x * 64 + threadIdx.x;
    if (i >= count) return;
    inner_finalize_group<NS>(groups + gidx[i], flags);
}

}  // namespace fk
}  // namespace ne
