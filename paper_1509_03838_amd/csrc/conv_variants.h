// Digit counts of the fused convolution and the set of kernel variants they
// call for (private to libne). Shared by the planner, which picks the digit
// counts of a group, and by the kernel translation units, which instantiate
// exactly the variants some group can need, so the two cannot disagree.
//
// A variant is (kernel class, slot count, LA, LB, shape):
//   kernel class 0: entangled groups, M = slots (M >= 3);
//   kernel class 1: plain and plain-same groups, M = slots;
//   kernel class 2: checksum groups (either datapath), M = slots - 1 data
//   streams + their sum.
#pragma once

#include <stdint.h>

namespace ne {

constexpr int kConvClassEntangled = 0;
constexpr int kConvClassPlain = 1;
constexpr int kConvClassChecksum = 2;

// Fewest balanced base-256 digits (each in [-128, 127]) that represent every
// integer in [-neg, pos]: L digits reach -128 R and 127 R, R = (256^L - 1)/255.
constexpr int digits_for(unsigned __int128 neg, unsigned __int128 pos)
{
    unsigned __int128 R = 0, p = 1;
    for (int L = 1; L <= 16; ++L) {
        R += p;
        p *= 256;
        if (128 * R >= neg && 127 * R >= pos) return L;
    }
    return 17;
}

// Shift l of Table I's rule at word width w (l = ceil(w/M), k = w - (M-1) l,
// or l = k = floor(w/M) when k would be negative).
constexpr int table1_shift(int M, int w)
{
    int l = (w + M - 1) / M;
    if (w - (M - 1) * l < 0) l = w / M;
    return l;
}

constexpr int table1_shift64(int M) { return table1_shift(M, 64); }

// D of eq. (11) (M = 3) or eq. (13) (M > 3) at w = 32, the largest output
// magnitude groups in 32-bit words may produce (M in [3, 8]).
constexpr int64_t dmax_w32(int M)
{
    const int l = table1_shift(M, 32);
    int k = 32 - (M - 1) * l;
    if (k < 0) k = l;
    if (M == 3) return ((int64_t)1 << (l + k - 1)) - ((int64_t)1 << l);
    return ((int64_t)1 << ((M - 3) * l + k)) * (((int64_t)1 << (l - 1)) - 1);
}

struct DigitCounts {
    int la, lb;
    int sparse;  // 1: the taps' top digit is nonzero only for a sliver of their range
    int split;   // 1: data words split at bit l into two fields of la/2 digits each
    int l;       // split words: the field boundary (Table I's l of the datapath, <= 22)
};

// Variant shape index of a digit count: 0 plain digits, 1 sparse top tap
// digit, 2 data words split into two fields (the two never combine).
constexpr int conv_shape(const DigitCounts &d) { return d.sparse ? 1 : (d.split ? 2 : 0); }
constexpr int kConvShapes = 3;

// Balanced digits reach 127 * R on the positive side (R = (256^L - 1)/255),
// one step short of a power of two: taps of 16 bits need a third digit, but
// only for values above 127 * 257. When LB - 1 digits cover all but such a
// sliver (at most 1/32 of the values), the kernel runs the top digit plane
// only for the chunks of taps that need it.
constexpr int sparse_top_digit(int in_bits, int lb)
{
    if (lb < 2) return 0;
    const unsigned __int128 B = (unsigned __int128)1 << (in_bits - 1);
    unsigned __int128 R = 0, p = 1;
    for (int L = 1; L < lb; ++L) {
        R += p;
        p *= 256;
    }
    if (128 * R < B || 127 * R >= B - 1) return 0;
    return (B - 1 - 127 * R) * 32 <= 2 * B ? 1 : 0;
}

// Digits of the data words and of the taps of a convolution group whose
// inputs and taps lie in [-2^(b-1), 2^(b-1) - 1]. Entangled words
// c + 2^l c' (l of Table I at word width w) lie in (2^l + 1) times that
// range (plain-same groups use the same digit count on raw words, so that
// both modes run one datapath); the checksum stream in M times that range.
// mode: 0 entangled, 1 plain, 2 plain-same, 3 checksum, 4 checksum on the
// entangled datapath (the plan's modes).
//
// Split words (split = 1, allow_split): a word x is cut at bit l into
// lo = x - 2^l floor(x / 2^l + 1/2), the balanced low field, and
// hi = (x - lo) / 2^l, so x = lo + 2^l hi for every x; each field gets la/2
// balanced digits and the digit planes carry weights 256^a (lo) and
// 2^l 256^a (hi). An entangled word whose streams fit the lo field
// (|c| < 2^(l-1)) then needs the digits of two raw samples, not those of a
// word (2^l + 1) times wider: 4 instead of 5 for 12-bit samples at M = 3.
// It is chosen only where it needs fewer digit planes.
constexpr DigitCounts conv_digits(int mode, int M, int in_bits, int w = 64, bool allow_split = false)
{
    const unsigned __int128 B = (unsigned __int128)1 << (in_bits - 1);
    unsigned __int128 neg = B, pos = B - 1;
    const int lb = digits_for(B, B - 1);
    const DigitCounts narrow{0, lb, sparse_top_digit(in_bits, lb), 0, 0};
    if (mode == 0 || mode == 2 || mode == 4) {
        const int l = table1_shift(M < 3 ? 3 : M, w);
        const unsigned __int128 f = ((unsigned __int128)1 << l) + 1;
        int la = digits_for(neg * f, pos * f);
        // checksum on this datapath: the sum stream must fit it too
        if (mode == 4 && digits_for(neg * (unsigned)M, pos * (unsigned)M) > la)
            la = digits_for(neg * (unsigned)M, pos * (unsigned)M);
        if (allow_split && narrow.sparse == 0 && l <= 31) {
            // the lo field must hold every raw value (and the checksum sum)
            const unsigned __int128 fneg = mode == 4 ? neg * (unsigned)M : neg;
            const unsigned __int128 fpos = mode == 4 ? pos * (unsigned)M : pos;
            const unsigned __int128 half = (unsigned __int128)1 << (l - 1);
            const int fs = digits_for(fneg, fpos);
            if (fneg <= half && fpos < half && 2 * fs < la && 2 * fs <= 8)
                return DigitCounts{2 * fs, lb, 0, 1, l};
        }
        return DigitCounts{la, lb, narrow.sparse, 0, 0};
    }
    if (mode == 3) {
        neg *= (unsigned)M;
        pos *= (unsigned)M;
    }
    return DigitCounts{digits_for(neg, pos), lb, narrow.sparse, 0, 0};
}

// Widest inputs of a convolution group in 32-bit words: its worst case
// 2^(b-1) 2^(b-1) K (K >= 1) must stay within D (plain and checksum groups:
// within 2^31 - 1; M < 3 counts as 3).
constexpr int conv_w32_max_bits(int mode, int M)
{
    const int64_t lim = mode == 0 ? dmax_w32(M < 3 ? 3 : M) : (int64_t)0x7fffffff;
    int b = 1;
    while (b < 31 && ((int64_t)1 << (2 * b)) <= lim) ++b;  // (b+1)-bit inputs still fit
    return b;
}

constexpr int kConvModes = 5;
constexpr bool conv_checksum_mode(int mode) { return mode == 3 || mode == 4; }
constexpr int conv_class_of_mode(int mode)
{
    return mode == 0 ? 0 : (conv_checksum_mode(mode) ? 2 : 1);
}

// Slots of a group: M, or M + 1 with the checksum stream.
constexpr int conv_slots(int mode, int M) { return conv_checksum_mode(mode) ? M + 1 : M; }

// Whether some group of this kernel class and slot count, with inputs of
// 1..31 bits (64-bit words) or of the widths 32-bit words admit, uses digit
// counts (la, lb) with a sparse top tap digit or not.
constexpr bool conv_variant_needed(int kclass, int slots, int la, int lb, int shape)
{
    for (int mode = 0; mode < kConvModes; ++mode) {
        if (conv_class_of_mode(mode) != kclass) continue;
        const int M = conv_checksum_mode(mode) ? slots - 1 : slots;
        if (M < (mode == 0 ? 3 : (conv_checksum_mode(mode) ? 2 : 1))) continue;
        for (int b = 1; b <= 31; ++b) {
            const DigitCounts d = conv_digits(mode, M, b, 64, true);
            if (d.la == la && d.lb == lb && conv_shape(d) == shape) return true;
        }
        if (mode == 0 || mode == 2 || mode == 4) {  // 32-bit words: a shorter shift l
            const int bmax = conv_w32_max_bits(mode == 0 ? 0 : 1, M);
            for (int b = 1; b <= bmax; ++b) {
                const DigitCounts d = conv_digits(mode, M, b, 32, true);
                if (d.la == la && d.lb == lb && conv_shape(d) == shape) return true;
            }
        }
    }
    return false;
}

// Whether some group of this kernel class and slot count, with inputs of
// 1..max_bits bits, uses digit counts (la, lb) (any top-digit sparsity).
constexpr bool digits_needed(int kclass, int slots, int la, int lb, int max_bits)
{
    for (int mode = 0; mode < 4; ++mode) {  // (the matrix product has no mode 4)
        if (conv_class_of_mode(mode) != kclass) continue;
        const int M = mode == 3 ? slots - 1 : slots;
        if (M < (mode == 0 ? 3 : (mode == 3 ? 2 : 1)) || M > 8) continue;
        for (int b = 1; b <= max_bits; ++b) {
            const DigitCounts d = conv_digits(mode, M, b);
            if (d.la == la && d.lb == lb) return true;
        }
    }
    return false;
}

// Whether some matrix-product group of this kernel class and slot count,
// with values of 1..max_bits bits, takes split words of la / 2 digits per
// field and lb digits for the kernel matrix (entangled and plain-same).
constexpr bool gemm_split_needed(int kclass, int slots, int la, int lb, int max_bits)
{
    for (int mode = 0; mode < 3; ++mode) {
        if (conv_class_of_mode(mode) != kclass || mode == 1) continue;
        const int M = slots;
        if (M < (mode == 0 ? 3 : 1) || M > 8) continue;
        for (int b = 1; b <= max_bits; ++b) {
            const DigitCounts d = conv_digits(mode, M, b, 64, true);
            if (d.split && d.la == la && d.lb == lb) return true;
        }
    }
    return false;
}

// The single-launch executor (one persistent kernel per kernel class) holds
// a fixed menu of kernel bodies: the element-wise operations scale, add,
// inner product and permutation, and the convolution variants (linear,
// circular, cross-correlation) that groups of 3..8 data streams with
// samples and taps of 9..12 bits take, in the block-ring and per-wave-ring
// layouts. A plan whose groups fall outside the menu runs as separate
// launches.
constexpr int kSingleBitsLo = 9, kSingleBitsHi = 12;

constexpr bool single_conv_in_menu(int kclass, int slots, int la, int lb, int shape)
{
    for (int mode = 0; mode < kConvModes; ++mode) {
        if (conv_class_of_mode(mode) != kclass) continue;
        const int M = conv_checksum_mode(mode) ? slots - 1 : slots;
        if (M < 3 || M > 8) continue;
        for (int b = kSingleBitsLo; b <= kSingleBitsHi; ++b) {
            const DigitCounts d = conv_digits(mode, M, b, 64, true);
            if (d.la == la && d.lb == lb && conv_shape(d) == shape) return true;
        }
    }
    return false;
}

// Slot counts of the menu's kernel bodies: 3..8 data streams, + the checksum.
constexpr int single_slots_lo(int kclass) { return kclass == 2 ? 4 : 3; }
constexpr int single_slots_hi(int kclass) { return kclass == 2 ? 9 : 8; }

}  // namespace ne
