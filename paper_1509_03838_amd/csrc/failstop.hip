// Fail-stop identification by deadline (ne_wait_streams): the paper's
// failure model is a core that becomes unresponsive or late (Sec. I), and
// recovery assumes the unavailable stream is known (Sec. III-B). Here each
// entangled stream's operation runs as its own task on its own HIP stream
// and ends with a completion event; the host waits for the events until a
// deadline and names the one stream that missed it. ne_stream_delay models
// a slow core: a bounded wait enqueued before a stream's work.
#include <chrono>
#include <thread>

#include "ne_internal.h"

namespace {

// One lane spins on the 100 MHz real-time counter until `ticks` have
// passed (bounded by the caller's limit), sleeping between reads.
__global__ void k_delay(uint64_t ticks)
{
    if (threadIdx.x != 0) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (__builtin_amdgcn_s_memrealtime() - t0 < ticks) __builtin_amdgcn_s_sleep(127);
}

}  // namespace

extern "C" {

ne_status ne_stream_delay(int64_t microseconds, ne_stream stream)
{
    if (microseconds < 0 || microseconds > NE_MAX_DELAY_US) return NE_EINVAL;
    if (microseconds == 0) return NE_OK;
    hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, (hipStream_t)stream,
                       (uint64_t)microseconds * 100u);
    return ne::launch_status();
}

ne_status ne_wait_streams(int32_t M, void *const *events, int64_t deadline_us, int32_t *lost)
{
    if (M < 1 || M > NE_MAX_M || !events || !lost || deadline_us < 0) return NE_EINVAL;
    using clock = std::chrono::steady_clock;
    const auto end = clock::now() + std::chrono::microseconds(deadline_us);
    uint64_t pending = 0;  // bit m: stream m has not completed
    for (int m = 0; m < M; ++m) pending |= 1ull << m;
    for (;;) {
        for (int m = 0; m < M; ++m) {
            if (!((pending >> m) & 1)) continue;
            if (!events[m]) continue;  // never launched: it cannot complete
            const hipError_t e = hipEventQuery((hipEvent_t)events[m]);
            if (e == hipSuccess) {
                pending &= ~(1ull << m);
            } else if (e != hipErrorNotReady) {
                return ne::hip_fail(e);
            }
        }
        if (!pending || clock::now() >= end) break;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (!pending) {
        *lost = -1;
        return NE_OK;
    }
    if (pending & (pending - 1)) {  // two or more late: beyond what one redundant stream covers
        *lost = -1;
        return NE_ELATE;
    }
    *lost = __builtin_ctzll(pending);
    return NE_OK;
}

}  // extern "C"
