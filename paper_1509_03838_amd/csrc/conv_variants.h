// Digit counts of the fused convolution and the set of kernel variants they
// call for (private to libne). Shared by the planner, which picks the digit
// counts of a group, and by the kernel translation units, which instantiate
// exactly the variants some group can need, so the two cannot disagree.
//
// A variant is (kernel class, slot count, LA, LB):
//   kernel class 0: entangled groups, M = slots (M >= 3);
//   kernel class 1: plain and plain-same groups, M = slots;
//   kernel class 2: checksum groups, M = slots - 1 data streams + their sum.
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
};

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
// mode: 0 entangled, 1 plain, 2 plain-same, 3 checksum (the plan's modes).
constexpr DigitCounts conv_digits(int mode, int M, int in_bits, int w = 64)
{
    const unsigned __int128 B = (unsigned __int128)1 << (in_bits - 1);
    unsigned __int128 neg = B, pos = B - 1;
    if (mode == 0 || mode == 2) {
        const unsigned __int128 f = ((unsigned __int128)1 << table1_shift(M < 3 ? 3 : M, w)) + 1;
        neg *= f;
        pos *= f;
    } else if (mode == 3) {
        neg *= (unsigned)M;
        pos *= (unsigned)M;
    }
    const int lb = digits_for(B, B - 1);
    return DigitCounts{digits_for(neg, pos), lb, sparse_top_digit(in_bits, lb)};
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

constexpr int conv_class_of_mode(int mode) { return mode == 0 ? 0 : (mode == 3 ? 2 : 1); }

// Slots of a group: M, or M + 1 with the checksum stream.
constexpr int conv_slots(int mode, int M) { return mode == 3 ? M + 1 : M; }

// Whether some group of this kernel class and slot count, with inputs of
// 1..31 bits (64-bit words) or of the widths 32-bit words admit, uses digit
// counts (la, lb) with a sparse top tap digit or not.
constexpr bool conv_variant_needed(int kclass, int slots, int la, int lb, int sparse)
{
    for (int mode = 0; mode < 4; ++mode) {
        if (conv_class_of_mode(mode) != kclass) continue;
        const int M = mode == 3 ? slots - 1 : slots;
        if (M < (mode == 0 ? 3 : (mode == 3 ? 2 : 1))) continue;
        for (int b = 1; b <= 31; ++b) {
            const DigitCounts d = conv_digits(mode, M, b);
            if (d.la == la && d.lb == lb && d.sparse == sparse) return true;
        }
        if (mode == 0 || mode == 2) {  // 32-bit words: a shorter shift l
            const int bmax = conv_w32_max_bits(mode == 0 ? 0 : 1, M);
            for (int b = 1; b <= bmax; ++b) {
                const DigitCounts d = conv_digits(mode, M, b, 32);
                if (d.la == la && d.lb == lb && d.sparse == sparse) return true;
            }
        }
    }
    return false;
}

// Whether some group of this kernel class and slot count, with inputs of
// 1..max_bits bits, uses digit counts (la, lb) (any top-digit sparsity).
constexpr bool digits_needed(int kclass, int slots, int la, int lb, int max_bits)
{
    for (int mode = 0; mode < 4; ++mode) {
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

}  // namespace ne
