// Private declarations shared by the translation units of libne.
// Kernel argument blocks are passed by value in the kernarg segment; every
// pointer table is indexed either with compile-time indices (templated
// kernels) or with wave-uniform indices, so none of them is copied to
// scratch memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ne.h"

namespace ne {

constexpr int kMaxM = NE_MAX_M;

struct PtrsI32 {
    const int32_t *p[kMaxM];
};
struct PtrsCI64 {
    const int64_t *p[kMaxM];
};
struct PtrsI64 {
    int64_t *p[kMaxM];
};
struct PtrsW32 {
    int32_t *p[kMaxM];
};

// Records a failed HIP call for ne_last_hip_error() and returns NE_EHIP.
ne_status hip_fail(hipError_t e);
// Checks hipGetLastError() after a launch.
ne_status launch_status();
// The library's device flag word on the current device (ne_device_flags):
// kernels of the per-step calls OR NE_FLAG_* bits into it. Its address is
// looked up once per device; NULL if the lookup failed (the kernels then
// report nothing).
uint32_t *device_flag_word();
// Shape rules of one LSB operation (ne_lsb_apply): NE_OK, NE_EINVAL or
// NE_EUNSUP.
ne_status check_op_shape(int32_t op, int64_t n_in, const void *operand, int64_t n_operand,
                         int64_t n_out);

// A run of consecutive element-wise operations of a series (scale, add, sub,
// mul), optionally led by a permutation, applied in one pass over the
// entangled words: out[i] = op_k( ... op_1(in[p[i]] or in[i]) ...).
constexpr int kMaxSegmentOps = 8;
struct SegmentOp {
    int32_t op;
    int32_t pad_;
    const void *g;  // NE_OP_ADD / NE_OP_SUB: words of the stream width; NE_OP_MUL: int32
    int64_t s;      // NE_OP_SCALE
};
struct Segment {
    int32_t nops;
    int32_t perm;          // 1: gather at p[i] first
    const int32_t *p;
    // 0: stream t's input words are the plane in.p[t]; > 0: they are
    // interleaved in rows of that many words (stream t of position i at
    // in.p[0][i * rows + t]), so that a gather fetches every stream's word of
    // one position from one place
    int32_t rows;
    int32_t pad_;
    SegmentOp ops[kMaxSegmentOps];
};

// The run's operations on the word v of output position i (wrapping modulo
// 2^(8 sizeof W)).
template <typename W>
__device__ __forceinline__ W segment_ops(W v0, const Segment &seg, int64_t i)
{
    using U = typename std::make_unsigned<W>::type;
    U v = (U)v0;
    for (int k = 0; k < seg.nops; ++k) {
        const SegmentOp &o = seg.ops[k];
        switch (o.op) {
        case NE_OP_SCALE: v = v * (U)o.s; break;
        case NE_OP_ADD: v = v + (U)((const W *)o.g)[i]; break;
        case NE_OP_SUB: v = v - (U)((const W *)o.g)[i]; break;
        default: v = v * (U)(W)((const int32_t *)o.g)[i]; break;  // NE_OP_MUL
        }
    }
    return (W)v;
}

// The same run on the words of R streams at one position: every operand
// word is read once for all of them.
template <typename W, int R>
__device__ __forceinline__ void segment_ops_all(W (&v)[R], const Segment &seg, int64_t i)
{
    using U = typename std::make_unsigned<W>::type;
    for (int k = 0; k < seg.nops; ++k) {
        const SegmentOp &o = seg.ops[k];
        if (o.op == NE_OP_SCALE) {
#pragma unroll
            for (int t = 0; t < R; ++t) v[t] = (W)((U)v[t] * (U)o.s);
            continue;
        }
        const U g = o.op == NE_OP_MUL ? (U)(W)((const int32_t *)o.g)[i] : (U)((const W *)o.g)[i];
        if (o.op == NE_OP_ADD) {
#pragma unroll
            for (int t = 0; t < R; ++t) v[t] = (W)((U)v[t] + g);
        } else if (o.op == NE_OP_SUB) {
#pragma unroll
            for (int t = 0; t < R; ++t) v[t] = (W)((U)v[t] - g);
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) v[t] = (W)((U)v[t] * g);
        }
    }
}

// ------------------------------------------------------------- launchers
// All launchers assume validated arguments (the C-ABI layer checks them).

// eps_m = c_m + 2^l c_{m-1}; M in [3, kMaxM].
void launch_entangle(int M, int l, int64_t n, const PtrsI32 &c, const PtrsI64 &eps,
                     hipStream_t s);
void launch_entangle_inplace(int M, int l, int64_t n, const PtrsI64 &x, hipStream_t s);
void launch_entangle_operand(int l, int64_t n, const int32_t *g, int64_t *g_ent,
                             hipStream_t s);

// Recovery. `in` holds the M-1 available entangled outputs in the order
// delta_{r+1}, ..., delta_{r+M-1} (indices mod M); `out` receives
// d_{r+1}, ..., d_{r+M-1}, d_r in that order.
void launch_extract(int M, int l, int64_t n, const PtrsCI64 &in, const PtrsI64 &out,
                    hipStream_t s);
// Recovery fused into the last run of a series: slot t (t < M - 1) takes the
// words of stream r+1+t -- in.p[t], or, with entangle, entangled on load from
// the int32 streams (c.p[u] is stream r + u mod M: slot t's word is
// c.p[t + 1] + 2^l c.p[t]) -- applies the run, and the M outputs are
// recovered and written as launch_extract writes them; with seg.rows > 0 (no
// entangle) slot t's words are in.p[0][i * seg.rows + t]. A permutation index
// outside [0, n) reads nothing (the word is 0) and raises NE_FLAG_PERM_INDEX
// in err.
void launch_segment_extract(int M, int l, int64_t n, bool entangle, const PtrsCI64 &in,
                            const PtrsI32 &c, const Segment &seg, const PtrsI64 &out,
                            uint32_t *err, hipStream_t s);
// The first run of a series with the entanglement on load: slots 0..count-1
// (count = M, or M - 1 with a lost stream) entangled from the int32 streams
// as above, each stream's sample read once per position, the run applied,
// slot t's words written to y.p[t]. Permutation indices as above.
void launch_segment_entangle(int M, int l, int64_t n, int count, const PtrsI32 &c,
                             const Segment &seg, const PtrsI64 &y, uint32_t *err, hipStream_t s);

// Element-wise LSB operations on `count` int64 streams (already compacted to
// the active ones).
void launch_scale_i64(int count, int64_t n, const PtrsCI64 &x, int64_t s_val, const PtrsI64 &y,
                      hipStream_t s);
void launch_add_i64(int count, int64_t n, const PtrsCI64 &x, const int64_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_perm_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *p, const PtrsI64 &y,
                     hipStream_t s);
void launch_inner_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, const PtrsI64 &y,
                      hipStream_t s);
// Convolution kinds: full linear, circular of length n, full cross-correlation.
constexpr int kConvLinear = 0, kConvCircular = 1, kConvXcorr = 2;
void launch_conv_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                     const PtrsI64 &y, hipStream_t s, int kind = kConvLinear);
// The same, writing the `count` outputs of each position as one row:
// stream t's output i goes to rows[i * count + t].
void launch_conv_i64_rows(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                          int64_t *rows, hipStream_t s, int kind = kConvLinear);
void launch_sub_i64(int count, int64_t n, const PtrsCI64 &x, const int64_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_mul_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_outer_i64(int count, int64_t n, const PtrsCI64 &x, const int32_t *g, int64_t K,
                      const PtrsI64 &y, hipStream_t s);

// The same operations on raw int32 streams with int64 results.
void launch_scale_i32(int count, int64_t n, const PtrsI32 &x, int64_t s_val, const PtrsI64 &y,
                      hipStream_t s);
void launch_add_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_perm_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *p, const PtrsI64 &y,
                     hipStream_t s);
void launch_inner_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                      hipStream_t s);
void launch_conv_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, int64_t K,
                     const PtrsI64 &y, hipStream_t s, int kind = kConvLinear);
void launch_sub_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_mul_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, const PtrsI64 &y,
                    hipStream_t s);
void launch_outer_i32(int count, int64_t n, const PtrsI32 &x, const int32_t *g, int64_t K,
                      const PtrsI64 &y, hipStream_t s);

// One LSB operation on `count` int32 streams of 32-bit entangled words
// (modulo 2^32), shapes already checked; every operand is int32.
void launch_op32(int32_t op, int count, int64_t n_in, const PtrsI32 &x, const int32_t *operand,
                 int64_t n_operand, int64_t scalar, const PtrsW32 &y, int64_t n_out,
                 hipStream_t s);

// The series in one call in 32-bit words: as launch_segment_entangle and
// launch_segment_extract, words and outputs int32 modulo 2^32,
// M in [3, NE_MAX_M32]; launch_extract32 recovers in place as
// ne_extract_recover32 does (in: the M - 1 slots from r + 1 on).
void launch_segment_entangle32(int M, int l, int64_t n, int count, const PtrsI32 &c,
                               const Segment &seg, const PtrsW32 &y, uint32_t *err, hipStream_t s);
void launch_segment_extract32(int M, int l, int64_t n, bool entangle, const PtrsI32 &in,
                              const PtrsI32 &c, const Segment &seg, const PtrsW32 &out,
                              uint32_t *err, hipStream_t s);
void launch_extract32(int M, int l, int64_t n, const PtrsI32 &in, const PtrsW32 &out,
                      hipStream_t s);
// A convolution kind (NE_OP_CONV, NE_OP_CIRC, NE_OP_XCORR) in 32-bit words
// writing rows: stream t's output i at rows[i * count + t].
void launch_conv32_rows(int32_t op, int count, int64_t n_in, const PtrsI32 &x,
                        const int32_t *operand, int64_t n_operand, int64_t n_out, int32_t *rows,
                        hipStream_t s);

// Checksum method.
void launch_checksum(int M, int64_t n, const PtrsI32 &c, int64_t *rsum, hipStream_t s);
void launch_checksum_recover(int count, int64_t n, const PtrsCI64 &d, const int64_t *e,
                             int64_t *d_r, hipStream_t s);

}  // namespace ne
