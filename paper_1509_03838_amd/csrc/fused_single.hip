// The single-launch executor of one kernel class (-DNE_KCLASS=k): one
// persistent kernel runs a whole plan. Its grid holds as many blocks as the
// device keeps resident at once; every block takes work items from one
// queue (a device counter) in the plan's order and runs each with the kernel
// body of its variant: convolution strips, element-wise strips, permutation
// layout passes. The bodies are those of the per-variant kernels; the menu
// of bodies is fixed (single_conv_in_menu, the element-wise operations
// scale, add, inner product and permutation, 3..8 data streams).
//
// Work items that depend on others:
//   * a permutation's gathers read the rows its layout items write: every
//     layout item is queued before every gather item, a layout item counts
//     itself done once its rows are written, and a gather item first waits
//     (bounded) until its group's count is complete. A block only claims a
//     gather item after all layout items have been claimed, by blocks that
//     are running and never wait, so the wait ends;
//   * an inner product's partial sums come from all its items: the block
//     that completes the last one recovers the outputs.
// What one item hands to another crosses XCDs (each has its own L2). The
// partial sums are device-scope atomics, and an inner-product item waits for
// its own to complete before it counts itself done. A layout item (64K
// positions) waits until its rows have reached its XCD's L2, then one wave
// writes that L2 back (a device-scope release) before the count. The
// gathers read the rows with ordinary loads: the caches start every launch
// empty of them and no one reads a row before its group's count is
// complete, so no cache holds an older copy, and no reader invalidates a
// cache. (A device-scope fence per small item, on both sides, cost more
// than the work: every fence writes back or invalidates a whole L2.)
// The counters return to zero within each run (the last gather of a group,
// the recovering block, the last block to leave the queue), so a captured
// run can be replayed.
#include "conv_variants.h"
#include "fused_kernels.h"

#if !defined(NE_KCLASS)
#error "NE_KCLASS selects the kernel class of this translation unit"
#endif

#define NE_CAT2(a, b) a##b
#define NE_NAME(a, b) NE_CAT2(a, b)

namespace ne {

namespace {

constexpr int kLo = single_slots_lo(NE_KCLASS);
constexpr int kHi = single_slots_hi(NE_KCLASS);

// Bound of a gather item's wait for its group's layout items (iterations of
// about 0.5 us, 0.5 s in all): far above any layout pass, so that a broken
// count ends in a flag instead of a hang; once one wait has raised the flag,
// the others end at their next iteration.
constexpr uint32_t kMaxSpins = 1u << 20;

constexpr int sp_of(int shape) { return shape == 1 ? 1 : 0; }
constexpr int fs_of(int la, int shape) { return shape == 2 ? la / 2 : 0; }

template <int NS, int LA, int LB, int SH>
__device__ __forceinline__ void conv_body(const GroupDev *groups, const Item it, int layout,
                                          uint32_t *flags)
{
    if constexpr ((SH == 1 && LB < 2) || (SH == 2 && LA % 2 != 0)) {
        return;
    } else if constexpr (single_conv_in_menu(NE_KCLASS, NS, LA, LB, SH)) {
        if (layout == 1)
            fk::conv_item<LA, LB, NS, NE_KCLASS, 1, sp_of(SH), 4, fs_of(LA, SH)>(groups, it, flags);
        else
            fk::conv_item<LA, LB, NS, NE_KCLASS, 4, sp_of(SH), 4, fs_of(LA, SH)>(groups, it, flags);
    }
}

template <int NS, int LA, int LB>
__device__ __forceinline__ void conv_shape(const GroupDev *groups, const Item it, int shape,
                                           int layout, uint32_t *flags)
{
    switch (shape) {
    case 0: conv_body<NS, LA, LB, 0>(groups, it, layout, flags); break;
    case 1: conv_body<NS, LA, LB, 1>(groups, it, layout, flags); break;
    default: conv_body<NS, LA, LB, 2>(groups, it, layout, flags); break;
    }
}

template <int NS, int LA>
__device__ __forceinline__ void conv_lb(const GroupDev *groups, const Item it, int lb, int shape,
                                        int layout, uint32_t *flags)
{
    switch (lb) {
    case 1: conv_shape<NS, LA, 1>(groups, it, shape, layout, flags); break;
    case 2: conv_shape<NS, LA, 2>(groups, it, shape, layout, flags); break;
    case 3: conv_shape<NS, LA, 3>(groups, it, shape, layout, flags); break;
    default: conv_shape<NS, LA, 4>(groups, it, shape, layout, flags); break;
    }
}

template <int NS>
__device__ __forceinline__ void conv_la(const GroupDev *groups, const Item it, int la, int lb,
                                        int shape, int layout, uint32_t *flags)
{
    switch (la) {
    case 1: conv_lb<NS, 1>(groups, it, lb, shape, layout, flags); break;
    case 2: conv_lb<NS, 2>(groups, it, lb, shape, layout, flags); break;
    case 3: conv_lb<NS, 3>(groups, it, lb, shape, layout, flags); break;
    case 4: conv_lb<NS, 4>(groups, it, lb, shape, layout, flags); break;
    case 5: conv_lb<NS, 5>(groups, it, lb, shape, layout, flags); break;
    case 6: conv_lb<NS, 6>(groups, it, lb, shape, layout, flags); break;
    case 7: conv_lb<NS, 7>(groups, it, lb, shape, layout, flags); break;
    default: conv_lb<NS, 8>(groups, it, lb, shape, layout, flags); break;
    }
}

// Element-wise body of (operation, slots); the operation's extra steps in a
// single launch (the wait of a gather, the recovery of an inner product)
// around it.
template <int OP, int NS>
__device__ __forceinline__ void stream_body(const GroupDev *groups, const Item it, uint32_t *flags)
{
    if constexpr (NS < kLo || NS > kHi) {
        return;
    } else {
        const GroupDev *G = groups + it.g;
        const int tid = threadIdx.x;
        if constexpr (OP == NE_OP_PERM) {
            if (tid == 0) {
                const uint32_t need = (uint32_t)G->nsync[0];
                uint32_t spins = 0;
                while (__hip_atomic_load(G->sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       need) {
                    __builtin_amdgcn_s_sleep(16);
                    if (++spins == kMaxSpins) {
                        atomicOr(flags, kFlagStall);
                        break;
                    }
                    if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                        kFlagStall)
                        break;
                }
            }
            __syncthreads();
        }
        constexpr int VX = stream_positions_of(OP, NS) / stream_positions(NS);
        fk::stream_item<OP, NE_KCLASS, NS, VX>(groups, it, flags);
        if constexpr (OP == NE_OP_PERM) {
            __syncthreads();  // every wave's gathers are done
            if (tid == 0 &&
                atomicAdd(G->sync + 1, 1u) == (uint32_t)G->nsync[1] - 1u) {
                atomicExch(G->sync, 0u);  // the group's last gather: clear for the next run
                atomicExch(G->sync + 1, 0u);
            }
        }
        if constexpr (OP == NE_OP_INNER) {
            __shared__ uint32_t s_last;
            __builtin_amdgcn_s_waitcnt(0);  // this item's partial sums are added
            __syncthreads();
            if (tid == 0)
                s_last = atomicAdd(G->sync, 1u) == (uint32_t)G->nsync[0] - 1u;
            __syncthreads();
            if (s_last && tid == 0) {
                // every item's partial sums, read (and cleared) by device-scope exchanges
                fk::inner_finalize_group<NS, true>(G, flags);
                atomicExch(G->sync, 0u);
            }
        }
    }
}

template <int OP>
__device__ __forceinline__ void stream_ns(const GroupDev *groups, const Item it, int ns,
                                          uint32_t *flags)
{
    switch (ns) {
    case 3: stream_body<OP, 3>(groups, it, flags); break;
    case 4: stream_body<OP, 4>(groups, it, flags); break;
    case 5: stream_body<OP, 5>(groups, it, flags); break;
    case 6: stream_body<OP, 6>(groups, it, flags); break;
    case 7: stream_body<OP, 7>(groups, it, flags); break;
    case 8: stream_body<OP, 8>(groups, it, flags); break;
    default: stream_body<OP, 9>(groups, it, flags); break;
    }
}

__device__ __forceinline__ void run_task(const GroupDev *groups, const Task t, uint32_t *flags)
{
    const uint32_t cat = t.kind & 3u;
    const int ns = (int)((t.kind >> 2) & 15u);
    const Item it{t.g, t.strip};
    if (cat == kTaskConv) {
        const int la = (int)((t.kind >> 10) & 15u), lb = (int)((t.kind >> 14) & 7u);
        const int shape = (int)((t.kind >> 17) & 3u), layout = (int)((t.kind >> 19) & 3u);
        switch (ns) {
        case 3: conv_la<3>(groups, it, la, lb, shape, layout, flags); break;
        case 4: conv_la<4>(groups, it, la, lb, shape, layout, flags); break;
        case 5: conv_la<5>(groups, it, la, lb, shape, layout, flags); break;
        case 6: conv_la<6>(groups, it, la, lb, shape, layout, flags); break;
        case 7: conv_la<7>(groups, it, la, lb, shape, layout, flags); break;
        case 8: conv_la<8>(groups, it, la, lb, shape, layout, flags); break;
        default: conv_la<9>(groups, it, la, lb, shape, layout, flags); break;
        }
    } else if (cat == kTaskStream) {
        switch ((int)((t.kind >> 6) & 15u)) {
        case NE_OP_SCALE: stream_ns<NE_OP_SCALE>(groups, it, ns, flags); break;
        case NE_OP_ADD: stream_ns<NE_OP_ADD>(groups, it, ns, flags); break;
        case NE_OP_INNER: stream_ns<NE_OP_INNER>(groups, it, ns, flags); break;
        default: stream_ns<NE_OP_PERM>(groups, it, ns, flags); break;
        }
    } else {
        const GroupDev *G = groups + t.g;
        if (G->nslots <= 4)
            fk::interleave_item<4>(groups, it, (int)t.steps);
        else
            fk::interleave_item<8>(groups, it, (int)t.steps);
        __builtin_amdgcn_s_waitcnt(0);  // this wave's rows are in the L2
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the L2 written back
            atomicAdd(G->sync, 1u);
        }
    }
}

// (at least 2 waves per SIMD: the menu's heaviest bodies would otherwise
// take the whole register file)
__global__ __launch_bounds__(fk::kBlock, 2) void k_persistent(const GroupDev *__restrict__ groups,
                                                           const Task *__restrict__ tasks,
                                                           uint32_t ntasks, uint32_t *queue,
                                                           uint32_t *flags)
{
    __shared__ uint32_t s_task[2];
    const bool lead = threadIdx.x == 0;
    if (lead) s_task[0] = atomicAdd(queue, 1u);
    __syncthreads();
    // uniform: the item's descriptor fields go to scalar registers
    uint32_t i = __builtin_amdgcn_readfirstlane(s_task[0]);
    int buf = 1;
    while (i < ntasks) {
        // The next claim is in flight while this item runs. It comes later
        // in the queue than this item, so it is never a layout item that a
        // gather running here waits for.
        uint32_t next = 0;
        if (lead) next = atomicAdd(queue, 1u);
        run_task(groups, tasks[i], flags);
        if (lead) s_task[buf] = next;
        // also orders this item's LDS use before the next item's
        __syncthreads();
        i = __builtin_amdgcn_readfirstlane(s_task[buf]);
        buf ^= 1;
    }
    // the last block to leave clears the queue for the next run
    if (threadIdx.x == 0 && atomicAdd(queue + 1, 1u) == gridDim.x - 1u) {
        atomicExch(queue, 0u);
        atomicExch(queue + 1, 0u);
    }
}

void launch(const GroupDev *g, const Task *tasks, uint32_t ntasks, uint32_t *queue,
            uint32_t *flags, uint32_t grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(fk::kBlock), lds, s, g, tasks, ntasks, queue,
                       flags);
}

hipError_t prepare(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t blocks_per_cu(size_t lds, int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void *>(&k_persistent), fk::kBlock, lds);
}

const SingleKernel kernel{&launch, &prepare, &blocks_per_cu};

}  // namespace

const SingleKernel *NE_NAME(single_kernel_, NE_KCLASS)() { return &kernel; }

}  // namespace ne
