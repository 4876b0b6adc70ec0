// Batched executor (ne_plan_*): validation, digit-count choice, work-item
// construction and launch of the fused kernels.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "conv_variants.h"
#include "fused.h"
#include "ne_internal.h"

using namespace ne;

struct Bucket {
    int conv;             // 1: convolution kernel, 0: element-wise kernel
    int cls, la, lb;      // convolution: variant id (((class * 16 + slots) << 3) |
                          // (sparse top tap digit << 2) | LDS layout) and digits; element-wise: variant id
                          // ((op * 4 + class) * 16 + slots); layout pass: slot class
    const ConvKernel *ck; // convolution kernel variant
    StreamLaunch sk;      // element-wise kernel variant
    size_t lds;
    uint32_t first, count;  // range in the item array
};

struct ne_plan {
    int mode = 0;
    std::vector<GroupDev> host_groups;
    std::vector<Bucket> buckets;
    std::vector<Item> items;
    std::vector<uint32_t> inner;
    std::vector<Task> tasks;           // single launch: the work queue, in order
    std::vector<unsigned char> image;  // host copy of the device tables, uploaded verbatim
    size_t sz_groups = 0, sz_items = 0, sz_inner = 0, sz_acc = 0, sz_flags = 0, sz_rows = 0;
    size_t sz_tasks = 0, sz_sync = 0;
    std::vector<std::pair<uint32_t, size_t>> rows;  // permutation groups: (group, row offset)
    bool owns_arena = false;
    unsigned char *arena = nullptr;  // device: groups | items | inner idx | acc | flags
    GroupDev *d_groups = nullptr;
    Item *d_items = nullptr;
    uint32_t *d_inner = nullptr;
    uint32_t n_inner = 0;
    uint32_t *d_flags = nullptr;
    // single launch: its kernel, grid and LDS, the tasks, the queue (head,
    // blocks done) and the per-group counters
    const SingleKernel *single = nullptr;
    uint32_t single_grid = 0;
    size_t single_lds = 0;
    Task *d_tasks = nullptr;
    uint32_t *d_queue = nullptr;
    uint32_t *d_sync = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> branch;  // streams of the graph's parallel branches (capture only)
    std::vector<hipEvent_t> joins;    // their join events, then the fork event (kBranches + 1)
    ne_plan_stats stats{};
};

namespace {

constexpr int kConvStepsDefault = 4;
constexpr int kStreamStepsDefault = 4;
constexpr size_t kMaxLds = 160 * 1024;
constexpr size_t kBranches = 4;  // parallel branches of a captured run

inline bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// Blocks of a convolution variant that its registers let share a CU: a
// block's 4 waves take one wave slot on each SIMD, and a SIMD holds
// 512 / (VGPRs per lane, in granules of 8) waves. Read from the loaded
// kernel once per variant; 4 (the plan's cap) where no device can say.
int register_blocks(const ConvKernel *ck, int shape, int layout)
{
    static std::mutex mu;
    static std::map<std::tuple<const ConvKernel *, int, int>, int> cache;
    const auto key = std::make_tuple(ck, shape, layout);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int blocks = 4;
    hipFuncAttributes a{};
    if (ck->attributes[shape][layout] && ck->attributes[shape][layout](&a) == hipSuccess &&
        a.numRegs > 0)
        blocks = std::min(4, 512 / ((a.numRegs + 7) & ~7));
    else
        (void)hipGetLastError();
    cache[key] = blocks;
    return blocks;
}

}  // namespace

// Kernel variants whose LDS exceeds the default limit get it raised (once per
// plan creation; the plan tables are host-only until then).
static hipError_t plan_prepare(ne_plan *plan)
{
    if (plan->single) {
        // one launch of as many blocks as stay resident at once
        if (plan->single_lds > 64 * 1024) {
            const hipError_t e = plan->single->prepare(plan->single_lds);
            if (e != hipSuccess) return e;
        }
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = plan->single->blocks_per_cu(plan->single_lds, &per_cu);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
        plan->single_grid = (uint32_t)(per_cu * cus);
        return hipSuccess;
    }
    for (const Bucket &b : plan->buckets) {
        if (b.conv <= 0 || b.lds <= 64 * 1024) continue;
        const hipError_t e = b.ck->prepare[(b.cls >> 2) & 3][b.cls & 3](b.lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" {

static ne_status plan_build(const ne_group *groups, int32_t n_groups, int32_t mode,
                            const ne_tuning *tuning, ne_plan **out_plan)
{
    if (!out_plan || n_groups < 0 || (n_groups > 0 && !groups)) return NE_EINVAL;
    if (mode < kEntangled || mode > kChecksumSame) return NE_EINVAL;
    *out_plan = nullptr;
    const bool checksum = mode == kChecksum || mode == kChecksumSame;
    const int conv_steps = (tuning && tuning->conv_steps > 0) ? tuning->conv_steps : kConvStepsDefault;
    const int stream_steps =
        (tuning && tuning->stream_steps > 0) ? tuning->stream_steps : kStreamStepsDefault;
    if (conv_steps > 4096 || stream_steps > 4096) return NE_EINVAL;
    const int single_launch = tuning ? tuning->single_launch : 0;
    if (single_launch != 0 && single_launch != 1) return NE_EINVAL;
    const int kclass = conv_class_of_mode(mode);
    const SingleKernel *sk = single_launch ? single_kernel(kclass) : nullptr;
    if (single_launch && !sk) return NE_EUNSUP;

    ne_plan *plan = new (std::nothrow) ne_plan;
    if (!plan) return NE_ENOMEM;
    plan->mode = mode;
    plan->host_groups.resize(n_groups);
    std::vector<std::vector<Item>> per_group(n_groups);
    // bucket key -> items
    std::map<std::tuple<int, int, int, int>, std::vector<Item>> bucket_items;
    std::map<std::tuple<int, int, int, int>, size_t> bucket_lds;
    std::vector<uint32_t> inner_groups;
    size_t rows_bytes = 0;
    // single launch: tasks by queue section (layout passes; convolutions,
    // with their groups' work per strip for the longest-first order;
    // element-wise items; permutation gathers)
    std::vector<Task> t_layout, t_stream, t_perm;
    std::vector<std::pair<int64_t, std::vector<Task>>> t_conv;
    ne_plan_stats st{};
    st.groups = n_groups;

    for (int gi = 0; gi < n_groups; ++gi) {
        const ne_group &u = groups[gi];
        GroupDev &G = plan->host_groups[gi];
        memset(&G, 0, sizeof(G));
        auto fail = [&](ne_status s) {
            delete plan;
            return s;
        };
        const int minM = mode == kEntangled ? 3 : (checksum ? 2 : 1);
        if (u.M < minM || u.M > kFusedMaxM || u.n < 0 || u.in_bits < 1 || u.in_bits > 32)
            return fail(NE_EINVAL);
        if (u.lost < -1 || u.lost >= u.M) return fail(NE_EFAILIDX);
        if (u.steps < 0 || u.steps > 4096) return fail(NE_EINVAL);
        if (u.ring_waves != 0 && u.ring_waves != 1 && u.ring_waves != 4) return fail(NE_EINVAL);
        if (u.tap_copies != 0 && u.tap_copies != 1 && u.tap_copies != 4) return fail(NE_EINVAL);
        if (u.tap_copies == 1 && u.ring_waves == 1) return fail(NE_EINVAL);
        if (u.word_bits != 0 && u.word_bits != 32 && u.word_bits != 64) return fail(NE_EINVAL);
        const int w = u.word_bits == 32 ? 32 : 64;
        // the single launch balances its load through the queue: its items
        // are at least kSingleMinSteps long (each pays a claim and barriers)
        const int min_steps = sk ? kSingleMinSteps : 1;
        const int g_conv_steps = std::max(u.steps > 0 ? u.steps : conv_steps, min_steps);
        const int g_stream_steps = std::max(u.steps > 0 ? u.steps : stream_steps, min_steps);
        if (u.op < NE_OP_CONV || u.op > NE_OP_OUTER) return fail(NE_EUNSUP);
        const bool convlike = u.op == NE_OP_CONV || u.op == NE_OP_CIRC || u.op == NE_OP_XCORR;
        for (int m = 0; m < u.M; ++m) {
            if (!u.c[m] || !u.out[m] || !aligned(u.c[m], 16) || !aligned(u.out[m], 16))
                return fail(NE_EINVAL);
        }
        int64_t n_out;
        switch (u.op) {
        case NE_OP_CONV:
        case NE_OP_XCORR:
        case NE_OP_CIRC:
            if (u.n_operand < 1 || !u.operand || u.in_bits > 31) return fail(NE_EINVAL);
            n_out = u.op == NE_OP_CIRC ? u.n : (u.n == 0 ? 0 : u.n + u.n_operand - 1);
            break;
        case NE_OP_SCALE: n_out = u.n; break;
        case NE_OP_INNER: n_out = 1; break;
        case NE_OP_OUTER:
            if (u.n_operand < 0 || (u.n_operand > 0 && !u.operand)) return fail(NE_EINVAL);
            if (u.n_operand > 0 && u.n > INT64_MAX / u.n_operand) return fail(NE_EUNSUP);
            n_out = u.n * u.n_operand;
            break;
        default: n_out = u.n; break;
        }
        if (u.op == NE_OP_ADD || u.op == NE_OP_SUB || u.op == NE_OP_MUL || u.op == NE_OP_INNER ||
            u.op == NE_OP_PERM) {
            if (u.n_operand != u.n || (u.n > 0 && !u.operand)) return fail(NE_EINVAL);
        }
        if (u.operand && !aligned(u.operand, 16)) return fail(NE_EINVAL);
        if (u.op == NE_OP_PERM && u.n > INT32_MAX) return fail(NE_EUNSUP);

        // Worst-case output magnitude from the declared input range.
        const unsigned __int128 B = (unsigned __int128)1 << (u.in_bits - 1);
        unsigned __int128 bound = 0;
        const unsigned __int128 s_abs =
            (unsigned __int128)(u.scalar < 0 ? -(__int128)u.scalar : (__int128)u.scalar);
        switch (u.op) {
        case NE_OP_CONV:
        case NE_OP_CIRC:
        case NE_OP_XCORR: bound = B * B * (unsigned __int128)u.n_operand; break;
        case NE_OP_SCALE: bound = B * s_abs; break;
        case NE_OP_ADD:
        case NE_OP_SUB: bound = 2 * B; break;
        case NE_OP_MUL:
        case NE_OP_OUTER: bound = B * B; break;
        case NE_OP_INNER: bound = B * B * (unsigned __int128)(u.n > 0 ? u.n : 1); break;
        case NE_OP_PERM: bound = B; break;
        }
        int l = 0;
        int64_t D = 0;
        if (mode == kEntangled) {
            int32_t ll, kk;
            if (ne_params(u.M, w, &ll, &kk, &D) != NE_OK) return fail(NE_ERANGE);
            l = ll;
            if (bound > (unsigned __int128)D) return fail(NE_ERANGE);
        } else {
            const unsigned __int128 lim = ((unsigned __int128)1 << (w - 1)) - 1;
            const unsigned __int128 chk = checksum ? bound * (unsigned)u.M : bound;
            if (chk > lim) return fail(NE_ERANGE);
        }

        G.op = u.op;
        G.M = u.M;
        G.mode = checksum ? kChecksum : mode;  // the kernels run either checksum datapath alike
        G.lost = u.lost >= 0 ? 1 : 0;
        G.r = u.lost >= 0 ? u.lost : 0;
        G.l = l;
        G.nslots = checksum ? u.M + 1 : u.M;
        G.in_lo = u.in_bits == 32 ? INT32_MIN : -(int32_t)((int64_t)1 << (u.in_bits - 1));
        G.in_hi = u.in_bits == 32 ? INT32_MAX : (int32_t)(((int64_t)1 << (u.in_bits - 1)) - 1);
        G.n = u.n;
        G.K = (convlike || u.op == NE_OP_OUTER) ? u.n_operand : 0;
        G.out32 = w == 32;
        G.kind = u.op == NE_OP_CIRC ? kConvCircular : (u.op == NE_OP_XCORR ? kConvXcorr : kConvLinear);
        G.n_out = n_out;
        G.scalar = u.scalar;
        G.skip = G.lost ? (mode == kEntangled ? u.M - 1 : G.r) : -1;
        for (int t = 0; t < u.M; ++t) {
            const int m = mode == kEntangled ? (G.r + 1 + t) % u.M : t;
            G.c[t] = u.c[m];
            G.out[t] = (int64_t *)u.out[m];
        }
        G.operand = u.operand;
        const int cls = G.nslots <= 4 ? 0 : 1;

        // Algorithmic traffic and work of one run.
        st.in_bytes += (int64_t)u.M * u.n * 4 + (u.op == NE_OP_SCALE ? 0 : u.n_operand * 4);
        st.out_bytes += (int64_t)u.M * n_out * (w / 8);
        st.out_samples += (int64_t)u.M * n_out;
        if (convlike) st.macs += (int64_t)u.M * (u.op == NE_OP_CIRC ? n_out : u.n) * u.n_operand;
        if (u.op == NE_OP_MUL) st.macs += (int64_t)u.M * u.n;
        if (u.op == NE_OP_OUTER) st.macs += (int64_t)u.M * n_out;
        if (u.op == NE_OP_INNER) st.macs += (int64_t)u.M * u.n;

        if (n_out == 0) continue;
        if (convlike) {
            const DigitCounts dc = conv_digits(mode, u.M, u.in_bits, w, true);
            const int la = dc.la, lb = dc.lb, shape = conv_shape(dc);
            if (la > kLimbsA || lb > kLimbsB) return fail(NE_EUNSUP);
            G.la = la;
            G.lb = lb;
            G.nch = (int)((u.n_operand + 15 + 63) / 64);
            G.kp = 64 * G.nch - 16;
            // digits per field: a split word's pairs of one weight come from
            // one field
            const int fa = dc.split ? la / 2 : la;
            if (dc.split) {
                // the field boundary is the datapath's shift l in every mode
                // (groups of fewer than 3 streams take M = 3's)
                G.l = dc.l;
                // each field's whole digit sum fits in int32 when its
                // convolution does: |field| <= M 2^(b-1) (the checksum sum),
                // |taps| <= 2^(b-1), K taps
                const unsigned __int128 field = checksum ? B * (unsigned)u.M : B;
                G.acc16 = field * B * (unsigned __int128)u.n_operand < ((unsigned __int128)1 << 31);
            } else {
                // Neighbouring digit sums merge in int32 when
                // |acc_s| + 256 |acc_{s+1}| < 2^31, |acc_s| <= min(la, lb) 64 nch 2^14.
                G.acc16 = (int64_t)257 * std::min(la, lb) * 64 * G.nch * 16384 < ((int64_t)1 << 31);
            }
            G.steps = g_conv_steps;
            // int32 accumulation: a digit product is at most 2^14, summed over
            // 64 nch inputs and at most min(fa, lb) digit pairs per shift.
            if ((int64_t)64 * G.nch * std::min(fa, lb) * 16384 >= ((int64_t)1 << 31))
                return fail(NE_EUNSUP);
            const int nplanes = G.nslots;
            // LDS: tap-digit planes | digit-plane rings (one per block, or
            // one per wave with a window of 256 + kp each) | raw int32
            // staging of one step (the prefetch, below). Layouts: 0 block
            // ring, 4 tap copies; 1 per-wave rings, 4 copies; 2 block ring,
            // one copy.
            auto ring_lds = [&](int layout) {
                const int gw = conv_layout_waves(layout);
                return conv_tap_lds(G.nch, lb, conv_layout_copies(layout)) +
                       (size_t)(4 / gw) * nplanes * (la | 1) * (size_t)(256 * gw + G.kp);
            };
            // Blocks of this variant that can share a CU (bound by LDS and
            // by registers), with the raw-input prefetch buffer (M x 4 KiB)
            // when it costs no block.
            const ConvKernel *ck = conv_kernel(kclass, G.nslots, la, lb);
            if (!ck || !ck->launch[shape][0]) return fail(NE_EUNSUP);
            const size_t raw = (size_t)u.M * 4096;
            auto fit = [&](int layout, bool dma) {
                const size_t b = ring_lds(layout) + (dma ? raw : 0);
                if (b > kMaxLds) return (size_t)0;
                return std::min<size_t>(register_blocks(ck, shape, layout), kMaxLds / b);
            };
            auto use_dma = [&](int layout) {
                return g_conv_steps > 1 && fit(layout, true) >= fit(layout, false);
            };
            auto blocks = [&](int layout) { return fit(layout, use_dma(layout)); };
            // A block ring keeps 4 tap copies unless one copy fits more
            // blocks (or is the only fit); per-wave rings (no barriers) win
            // ties with block rings.
            auto block_ring = [&]() {
                if (u.tap_copies == 4) return 0;
                if (u.tap_copies == 1) return 2;
                return blocks(2) > blocks(0) ? 2 : 0;
            };
            int layout;
            if (u.ring_waves == 1 || (u.ring_waves == 0 && u.tap_copies != 1)) {
                layout = 1;
                if (u.ring_waves == 0 && blocks(block_ring()) > blocks(1)) layout = block_ring();
            } else {
                layout = block_ring();
            }
            if (blocks(layout) == 0) return fail(NE_EUNSUP);
            const int gw = conv_layout_waves(layout);
            G.ring_waves = gw;
            G.ring = 256 * gw + G.kp;
            G.dma = use_dma(layout);
            const size_t lds = ring_lds(layout) + (G.dma ? raw : 0);
            const int64_t strip = (int64_t)g_conv_steps * kConvTile;
            const int64_t nstrips = (n_out + strip - 1) / strip;
            auto key = std::make_tuple(1, ((kclass * 16 + G.nslots) << 4) | (shape << 2) | layout,
                                       la, lb);
            auto &v = bucket_items[key];
            for (int64_t s = 0; s < nstrips; ++s) v.push_back(Item{(uint32_t)gi, (uint32_t)s});
            bucket_lds[key] = std::max(bucket_lds[key], lds);
            if (sk) {
                if (layout > 1 || !single_conv_in_menu(kclass, G.nslots, la, lb, shape))
                    return fail(NE_EUNSUP);
                const uint32_t kind = task_kind(kTaskConv, G.nslots, u.op, la, lb, shape, layout);
                std::vector<Task> ts;
                for (int64_t s = 0; s < nstrips; ++s) ts.push_back(Task{kind, (uint32_t)gi, (uint32_t)s, 0});
                t_conv.emplace_back(strip * 64 * G.nch * la * lb, std::move(ts));
            }
            const int64_t slots_run = G.nslots - G.lost;
            // (a sparse top tap digit runs only where the taps need it: that
            // data-dependent part is not counted)
            st.mfma_macs += slots_run * nstrips * g_conv_steps * (int64_t)kConvTile * 64 * G.nch *
                            la * (lb - dc.sparse);
            st.limb_macs += slots_run * (u.op == NE_OP_CIRC ? n_out : u.n) * u.n_operand * la *
                            (lb - dc.sparse);
        } else {
            // element-wise kernel: kStreamV* positions per lane, `stream_steps` steps
            G.steps = g_stream_steps;
            const int64_t strip = (int64_t)g_stream_steps * 256 * stream_positions_of(u.op, G.nslots);
            // (the outer product's lanes run over its n K outputs)
            const int64_t nit = u.op == NE_OP_OUTER ? n_out : u.n;
            const int64_t nstrips = (nit + strip - 1) / strip;
            if (nstrips > ((int64_t)1 << 24)) return fail(NE_EUNSUP);  // work-item table size
            if (!stream_kernel(u.op, kclass, G.nslots)) return fail(NE_EUNSUP);
            if (sk) {
                if ((u.op != NE_OP_SCALE && u.op != NE_OP_ADD && u.op != NE_OP_INNER &&
                     u.op != NE_OP_PERM) ||
                    G.nslots < single_slots_lo(kclass) || G.nslots > single_slots_hi(kclass))
                    return fail(NE_EUNSUP);
                // an inner product's last item recovers it: at least one item
                const int64_t nt = u.op == NE_OP_INNER ? std::max<int64_t>(nstrips, 1) : nstrips;
                const uint32_t kind = task_kind(kTaskStream, G.nslots, u.op, 0, 0, 0, 0);
                auto &dst = u.op == NE_OP_PERM ? t_perm : t_stream;
                for (int64_t s = 0; s < nt; ++s) dst.push_back(Task{kind, (uint32_t)gi, (uint32_t)s, 0});
                if (u.op == NE_OP_INNER) G.nsync[0] = (int32_t)nt;
                if (u.op == NE_OP_PERM) G.nsync[1] = (int32_t)nt;
            }
            auto key = std::make_tuple(0, (u.op * 4 + kclass) * 16 + G.nslots, 0, 0);
            auto &v = bucket_items[key];
            for (int64_t s = 0; s < nstrips; ++s) v.push_back(Item{(uint32_t)gi, (uint32_t)s});
            if (u.op == NE_OP_INNER) inner_groups.push_back((uint32_t)gi);
            if (u.op == NE_OP_PERM && u.n > 0) {
                // interleaved rows (4 or 8 int32 per position) in the arena,
                // written by a layout pass launched before the element-wise kernels
                const size_t rw = cls == 0 ? 4 : 8;
                plan->rows.push_back({(uint32_t)gi, rows_bytes});
                rows_bytes += ((size_t)u.n * rw * 4 + 255) & ~(size_t)255;
                const int64_t istrip = (int64_t)g_stream_steps * kInterleaveStep;
                auto &iv = bucket_items[std::make_tuple(-1, cls, 0, 0)];
                const int64_t nlayout = (u.n + istrip - 1) / istrip;
                for (int64_t s = 0; s < nlayout; ++s)
                    iv.push_back(Item{(uint32_t)gi, (uint32_t)s});
                if (sk) {
                    // larger layout items: each ends with an L2 write-back
                    const uint32_t kind = task_kind(kTaskLayout, G.nslots, u.op, 0, 0, 0, 0);
                    const int64_t lstrip = (int64_t)kSingleLayoutSteps * kInterleaveStep;
                    const int64_t nl = (u.n + lstrip - 1) / lstrip;
                    for (int64_t s = 0; s < nl; ++s)
                        t_layout.push_back(
                            Task{kind, (uint32_t)gi, (uint32_t)s, (uint32_t)kSingleLayoutSteps});
                    G.nsync[0] = (int32_t)nl;
                }
            }
        }
    }

    // Flatten buckets; items of a bucket keep group order, strips ascending.
    std::vector<Item> all_items;
    for (auto &kv : bucket_items) {
        Bucket b{};
        b.conv = std::get<0>(kv.first);
        b.cls = std::get<1>(kv.first);
        b.la = std::get<2>(kv.first);
        b.lb = std::get<3>(kv.first);
        b.lds = b.conv > 0 ? bucket_lds[kv.first] : 0;
        b.ck = b.conv > 0 ? conv_kernel((b.cls >> 4) / 16, (b.cls >> 4) % 16, b.la, b.lb) : nullptr;
        b.sk = b.conv == 0 ? stream_kernel(b.cls / 64, (b.cls / 16) % 4, b.cls % 16) : nullptr;
        b.first = (uint32_t)all_items.size();
        b.count = (uint32_t)kv.second.size();
        all_items.insert(all_items.end(), kv.second.begin(), kv.second.end());
        plan->buckets.push_back(b);
        st.lds_bytes = std::max<int64_t>(st.lds_bytes, (int64_t)b.lds);
    }
    plan->n_inner = (uint32_t)inner_groups.size();
    st.items = (int64_t)all_items.size();
    st.launches = (int64_t)plan->buckets.size() + (plan->n_inner ? 1 : 0);
    if (sk) {
        // The queue: layout passes; then the convolutions (most work per
        // strip first, a group's strips together) interleaved evenly with
        // the permutation gathers, so that the matrix-core work overlaps the
        // gathers' memory latency; then the other element-wise items.
        std::stable_sort(t_conv.begin(), t_conv.end(),
                         [](const auto &a, const auto &b) { return a.first > b.first; });
        std::vector<Task> conv;
        for (auto &c : t_conv) conv.insert(conv.end(), c.second.begin(), c.second.end());
        std::vector<Task> &q = plan->tasks;
        q = std::move(t_layout);
        size_t ic = 0, ip = 0;
        while (ic < conv.size() || ip < t_perm.size()) {
            // take from the list that is further behind its share
            const bool take_conv =
                ip >= t_perm.size() ||
                (ic < conv.size() && (double)ic * t_perm.size() <= (double)ip * conv.size());
            q.push_back(take_conv ? conv[ic++] : t_perm[ip++]);
        }
        q.insert(q.end(), t_stream.begin(), t_stream.end());
        if (q.size() > ((size_t)1 << 31)) {
            delete plan;
            return NE_EUNSUP;
        }
        plan->single = sk;
        for (const Bucket &b : plan->buckets) plan->single_lds = std::max(plan->single_lds, b.lds);
        st.items = (int64_t)q.size();
        st.launches = q.empty() ? 0 : 1;
    }

    // One device arena: groups | items | inner index | accumulators | flags.
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    plan->sz_groups = up(sizeof(GroupDev) * std::max(1, n_groups));
    plan->sz_items = up(sizeof(Item) * std::max<size_t>(1, all_items.size()));
    plan->sz_inner = up(sizeof(uint32_t) * std::max<size_t>(1, inner_groups.size()));
    plan->sz_acc = up(sizeof(uint64_t) * kMaxSlots * std::max<size_t>(1, inner_groups.size()));
    plan->sz_flags = 256;
    plan->sz_rows = rows_bytes;
    if (sk) {
        plan->sz_tasks = up(sizeof(Task) * std::max<size_t>(1, plan->tasks.size()));
        plan->sz_sync = up(256 + sizeof(uint32_t) * 2 * std::max(1, n_groups));
    }
    plan->items = std::move(all_items);
    plan->inner = std::move(inner_groups);
    plan->stats = st;
    *out_plan = plan;
    return NE_OK;
}

// Device tables (uploaded from the host image) and the whole arena (the
// tables, then the permutation rows, which the layout pass writes).
static size_t table_bytes(const ne_plan *p)
{
    return p->sz_groups + p->sz_items + p->sz_inner + p->sz_acc + p->sz_flags + p->sz_tasks +
           p->sz_sync;
}

static size_t plan_bytes(const ne_plan *p) { return table_bytes(p) + p->sz_rows; }

// Points the plan at its device arena and lays out the host image of the
// tables (accumulators and flags zero) for one verbatim upload.
static void plan_place(ne_plan *plan, unsigned char *arena)
{
    plan->arena = arena;
    unsigned char *p = arena;
    plan->d_groups = (GroupDev *)p;
    p += plan->sz_groups;
    plan->d_items = (Item *)p;
    p += plan->sz_items;
    plan->d_inner = (uint32_t *)p;
    p += plan->sz_inner;
    uint64_t *d_acc = (uint64_t *)p;
    p += plan->sz_acc;
    plan->d_flags = (uint32_t *)p;
    p += plan->sz_flags;
    if (plan->single) {
        // tasks | queue (head, blocks done; 256 bytes) | two counters per group
        plan->d_tasks = (Task *)p;
        p += plan->sz_tasks;
        plan->d_queue = (uint32_t *)p;
        plan->d_sync = (uint32_t *)(p + 256);
        p += plan->sz_sync;
        for (size_t gi = 0; gi < plan->host_groups.size(); ++gi)
            plan->host_groups[gi].sync = plan->d_sync + 2 * gi;
    }
    for (const auto &r : plan->rows) plan->host_groups[r.first].rows = (int32_t *)(p + r.second);
    for (size_t i = 0; i < plan->inner.size(); ++i)
        plan->host_groups[plan->inner[i]].acc = d_acc + kMaxSlots * i;
    plan->image.assign(table_bytes(plan), 0);
    unsigned char *h = plan->image.data();
    memcpy(h, plan->host_groups.data(), sizeof(GroupDev) * plan->host_groups.size());
    memcpy(h + plan->sz_groups, plan->items.data(), sizeof(Item) * plan->items.size());
    memcpy(h + plan->sz_groups + plan->sz_items, plan->inner.data(),
           sizeof(uint32_t) * plan->inner.size());
    if (plan->single)
        memcpy(h + plan->sz_groups + plan->sz_items + plan->sz_inner + plan->sz_acc + plan->sz_flags,
               plan->tasks.data(), sizeof(Task) * plan->tasks.size());
}

ne_status ne_plan_create(const ne_group *groups, int32_t n_groups, int32_t mode,
                         const ne_tuning *tuning, ne_plan **out_plan)
{
    ne_plan *plan = nullptr;
    ne_status st = plan_build(groups, n_groups, mode, tuning, &plan);
    if (st != NE_OK) return st;
    hipError_t e = plan_prepare(plan);
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(e);
    }
    unsigned char *arena = nullptr;
    e = hipMalloc((void **)&arena, plan_bytes(plan));
    if (e != hipSuccess) {
        delete plan;
        (void)hipGetLastError();
        return NE_ENOMEM;
    }
    plan->owns_arena = true;
    plan_place(plan, arena);
    e = hipMemcpy(arena, plan->image.data(), plan->image.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ne_plan_destroy(plan);
        return hip_fail(e);
    }
    *out_plan = plan;
    return NE_OK;
}

ne_status ne_plan_workspace_size(const ne_group *groups, int32_t n_groups, int32_t mode,
                                 const ne_tuning *tuning, size_t *bytes)
{
    if (!bytes) return NE_EINVAL;
    ne_plan *plan = nullptr;
    ne_status st = plan_build(groups, n_groups, mode, tuning, &plan);
    if (st != NE_OK) return st;
    *bytes = plan_bytes(plan);
    delete plan;
    return NE_OK;
}

ne_status ne_plan_create_in(const ne_group *groups, int32_t n_groups, int32_t mode,
                            const ne_tuning *tuning, void *workspace, size_t workspace_bytes,
                            ne_stream stream, ne_plan **out_plan)
{
    if (!workspace || ((uintptr_t)workspace & 255u)) return NE_EINVAL;
    ne_plan *plan = nullptr;
    ne_status st = plan_build(groups, n_groups, mode, tuning, &plan);
    if (st != NE_OK) return st;
    if (plan_bytes(plan) > workspace_bytes) {
        delete plan;
        return NE_EINVAL;
    }
    hipError_t e = plan_prepare(plan);
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(e);
    }
    plan_place(plan, (unsigned char *)workspace);
    e = hipMemcpyAsync(workspace, plan->image.data(), plan->image.size(),
                                  hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(e);
    }
    *out_plan = plan;
    return NE_OK;
}

static void launch_bucket(const ne_plan *plan, const Bucket &b, hipStream_t s)
{
    if (b.count == 0) return;
    if (b.conv < 0)
        fused_interleave_launch(b.cls, plan->d_groups, plan->d_items + b.first, b.count, s);
    else if (b.conv)
        b.ck->launch[(b.cls >> 2) & 3][b.cls & 3](plan->d_groups, plan->d_items + b.first, b.count,
                                                  plan->d_flags, b.lds, s);
    else
        b.sk(plan->d_groups, plan->d_items + b.first, b.count, plan->d_flags, s);
}

static void launch_single(const ne_plan *plan, hipStream_t s)
{
    if (plan->tasks.empty()) return;
    plan->single->launch(plan->d_groups, plan->d_tasks, (uint32_t)plan->tasks.size(),
                         plan->d_queue, plan->d_flags, plan->single_grid, plan->single_lds, s);
}

ne_status ne_plan_run(ne_plan *plan, ne_stream stream)
{
    if (!plan) return NE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (plan->single) {
        launch_single(plan, s);
        return launch_status();
    }
    for (const Bucket &b : plan->buckets) launch_bucket(plan, b, s);
    if (plan->n_inner)
        fused_inner_finalize(plan->d_groups, plan->d_inner, plan->n_inner, plan->d_flags, s);
    return launch_status();
}

// The captured form of a run: the launches spread over up to kBranches
// parallel branches of the graph (they touch disjoint groups; running them
// side by side fills the tail of one with the next), then the inner-product
// recovery. A permutation layout pass and the permutation launches that read
// its rows form one chain on one branch.
static ne_status capture_branches(ne_plan *plan, hipStream_t s)
{
    if (plan->single) {
        launch_single(plan, s);
        return launch_status();
    }
    std::vector<std::vector<const Bucket *>> chains;
    int chain_of_cls[2] = {-1, -1};
    for (const Bucket &b : plan->buckets) {  // layout passes sort first
        if (b.count == 0) continue;
        if (b.conv < 0) {
            chain_of_cls[b.cls] = (int)chains.size();
            chains.push_back({&b});
        } else if (b.conv == 0 && b.cls / 64 == NE_OP_PERM) {
            const int c = chain_of_cls[(b.cls % 16) <= 4 ? 0 : 1];
            if (c >= 0)
                chains[c].push_back(&b);
            else
                chains.push_back({&b});
        } else {
            chains.push_back({&b});
        }
    }
    const int nb = (int)std::min<size_t>(plan->branch.size(), chains.size());
    if (nb <= 1) {
        for (const auto &ch : chains)
            for (const Bucket *b : ch) launch_bucket(plan, *b, s);
    } else {
        hipError_t e = hipSuccess;
        // longest chain first onto the least loaded branch (cost ~ items)
        auto cost = [](const std::vector<const Bucket *> &ch) {
            double c = 0;
            for (const Bucket *b : ch) c += (double)b->count * (b->conv > 0 ? 4.0 : 1.0);
            return c;
        };
        std::vector<int> order(chains.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::sort(order.begin(), order.end(),
                  [&](int x, int y) { return cost(chains[x]) > cost(chains[y]); });
        std::vector<double> load(nb, 0.0);
        std::vector<std::vector<int>> lanes(nb);
        for (int ci : order) {
            const int i = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            lanes[i].push_back(ci);
            load[i] += cost(chains[ci]);
        }
        e = hipEventRecord(plan->joins[kBranches], s);  // fork
        for (int i = 0; i < nb && e == hipSuccess; ++i) {
            e = hipStreamWaitEvent(plan->branch[i], plan->joins[kBranches], 0);
            for (int ci : lanes[i])
                for (const Bucket *b : chains[ci]) launch_bucket(plan, *b, plan->branch[i]);
            if (e == hipSuccess) e = hipEventRecord(plan->joins[i], plan->branch[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->joins[i], 0);  // join
        }
        if (e != hipSuccess) return hip_fail(e);
    }
    if (plan->n_inner)
        fused_inner_finalize(plan->d_groups, plan->d_inner, plan->n_inner, plan->d_flags, s);
    return launch_status();
}

ne_status ne_plan_capture(ne_plan *plan, ne_stream stream)
{
    if (!plan || !stream) return NE_EINVAL;  // the null stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    if (plan->exec) {
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    // branch streams and their events, created before the capture begins
    size_t nwork = 0;
    if (!plan->single)
        for (const Bucket &b : plan->buckets) nwork += b.count > 0;
    hipError_t e = hipSuccess;
    if (nwork > 1) {
        while (plan->branch.size() < kBranches && e == hipSuccess) {
            hipStream_t a = nullptr;
            e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
            if (e == hipSuccess) plan->branch.push_back(a);
        }
        while (plan->joins.size() < kBranches + 1 && e == hipSuccess) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) plan->joins.push_back(ev);
        }
        if (e != hipSuccess) return hip_fail(e);
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e);
    ne_status st = capture_branches(plan, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != NE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e);
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e);
    }
    plan->graph = g;
    return NE_OK;
}

ne_status ne_plan_launch(ne_plan *plan, ne_stream stream)
{
    if (!plan) return NE_EINVAL;
    if (!plan->exec) return ne_plan_run(plan, stream);
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    return e == hipSuccess ? NE_OK : hip_fail(e);
}

ne_status ne_plan_flags(ne_plan *plan, uint32_t *flags, int32_t clear)
{
    if (!plan || !flags) return NE_EINVAL;
    hipError_t e = hipMemcpy(flags, plan->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (clear) {
        const uint32_t z = 0;
        e = hipMemcpy(plan->d_flags, &z, sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
    }
    return NE_OK;
}

ne_status ne_plan_stats_get(const ne_plan *plan, ne_plan_stats *stats)
{
    if (!plan || !stats) return NE_EINVAL;
    *stats = plan->stats;
    return NE_OK;
}

ne_status ne_plan_destroy(ne_plan *plan)
{
    if (!plan) return NE_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->arena && plan->owns_arena) (void)hipFree(plan->arena);
    for (hipEvent_t ev : plan->joins) (void)hipEventDestroy(ev);
    for (hipStream_t a : plan->branch) (void)hipStreamDestroy(a);
    delete plan;
    return NE_OK;
}

}  // extern "C"
