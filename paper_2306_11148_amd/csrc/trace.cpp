// Kernel timing: event pairs around library launches, folded on request.
#include <atomic>
#include <mutex>
#include <vector>

#include "moa_internal.h"

namespace moa {
namespace {

struct Pending {
    int32_t kernel;
    hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_spare;
int64_t g_launches[MOA_K_COUNT];
double g_ms[MOA_K_COUNT];

hipEvent_t take_event() {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_spare.empty()) {
            hipEvent_t e = g_spare.back();
            g_spare.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

TraceScope::TraceScope(int32_t kernel, hipStream_t stream) : kernel_(kernel), stream_(stream) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream_, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
        return;   // no timing events inside graph captures
    start_ = take_event();
    if (start_ && hipEventRecord(start_, stream_) != hipSuccess) {
        (void)hipEventDestroy(start_);
        start_ = nullptr;
    }
}

TraceScope::~TraceScope() {
    if (!start_) return;
    hipEvent_t stop = take_event();
    if (!stop || hipEventRecord(stop, stream_) != hipSuccess) {
        (void)hipEventDestroy(start_);
        if (stop) (void)hipEventDestroy(stop);
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({kernel_, start_, stop});
}

}  // namespace moa

using namespace moa;

extern "C" {

moa_status moa_trace_enable(int32_t on) {
    g_on.store(on != 0);
    return MOA_OK;
}

moa_status moa_trace_read(moa_trace_stat *out, int32_t capacity, int32_t *count, int32_t reset) {
    if (!count || capacity < 0 || (capacity > 0 && !out)) return fail(MOA_ERR_INVALID, "bad arguments");
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<Pending> keep;
    for (const Pending &p : g_pending) {
        float ms = 0.0f;
        const hipError_t e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e == hipErrorNotReady) {
            keep.push_back(p);
            continue;
        }
        if (e == hipSuccess && p.kernel > 0 && p.kernel < MOA_K_COUNT) {
            g_launches[p.kernel] += 1;
            g_ms[p.kernel] += ms;
        }
        g_spare.push_back(p.start);
        g_spare.push_back(p.stop);
    }
    g_pending.swap(keep);
    int32_t n = 0;
    for (int k = 1; k < MOA_K_COUNT; ++k) {
        if (g_launches[k] == 0) continue;
        if (n < capacity) out[n] = {k, 0, g_launches[k], g_ms[k]};
        ++n;
    }
    *count = n < capacity ? n : capacity;
    if (reset)
        for (int k = 0; k < MOA_K_COUNT; ++k) {
            g_launches[k] = 0;
            g_ms[k] = 0.0;
        }
    return MOA_OK;
}

}  // extern "C"
