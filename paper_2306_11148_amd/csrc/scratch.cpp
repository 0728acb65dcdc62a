// Scratch memory of one call (conditioned operands, exponents, member tables).
//
// Device buffers are cached and reused. A cached buffer is handed to a call on
// the stream that used it last at once (stream order protects the earlier
// use), or to a call on another stream once the event recorded after its last
// use has completed; no call ever waits for another stream. Sizes are rounded
// up to powers of two (at least 1 MiB) so that a buffer fits later requests of
// similar size; new device memory is allocated only when no cached buffer
// fits, and idle buffers are released when the cache of a device would exceed
// kCacheBytes. Acquire and release are host operations of a few
// microseconds; the stream-ordered allocator's free costs tens to hundreds of
// microseconds per call on this runtime, which dominated small products and
// the serving loop. During stream capture the stream-ordered allocator is
// used instead, so that the allocation and free become graph nodes.
#include <mutex>
#include <vector>

#include "moa_internal.h"

namespace moa {
namespace {

constexpr int64_t kMinBucket = int64_t(1) << 20;
constexpr int64_t kCacheBytes = int64_t(64) << 30;   // per device

struct Buf {
    void *ptr = nullptr;
    int64_t bytes = 0;
    int dev = 0;
    hipEvent_t done = nullptr;          // recorded after the last use
    hipStream_t last = nullptr;         // stream of the last use
    bool busy = false;                  // handed out, not yet released
    bool used = false;                  // `done` has been recorded at least once
};

std::mutex g_mu;
std::vector<Buf> g_bufs;

int64_t bucket(int64_t bytes) {
    int64_t b = kMinBucket;
    while (b < bytes) b <<= 1;
    return b;
}

bool idle(const Buf &b) { return !b.busy && (!b.used || hipEventQuery(b.done) == hipSuccess); }

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

}  // namespace

moa_status scratch_alloc(void **ptr, int64_t bytes, hipStream_t stream) {
    *ptr = nullptr;
    if (bytes <= 0) return MOA_OK;
    hipError_t e;
    if (capturing(stream)) {
        e = hipMallocAsync(ptr, (size_t)bytes, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(MOA_ERR_NOMEM, "scratch of %lld bytes: %s", (long long)bytes, hipGetErrorString(e));
        }
        return MOA_OK;
    }
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    const int64_t want = bucket(bytes);
    std::vector<void *> drop;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        // smallest fitting buffer that this stream may use now
        int best = -1;
        for (int k = 0; k < (int)g_bufs.size(); ++k) {
            const Buf &b = g_bufs[k];
            if (b.dev != dev || b.busy || b.bytes < bytes) continue;
            if (best >= 0 && g_bufs[best].bytes <= b.bytes) continue;
            if ((b.used && b.last == stream) || idle(b)) best = k;
        }
        if (best >= 0) {
            g_bufs[best].busy = true;
            *ptr = g_bufs[best].ptr;
            return MOA_OK;
        }
        // make room: release idle buffers while the cache would exceed its cap
        int64_t held = 0;
        for (const Buf &b : g_bufs)
            if (b.dev == dev) held += b.bytes;
        for (int k = 0; k < (int)g_bufs.size() && held + want > kCacheBytes;) {
            Buf &b = g_bufs[k];
            if (b.dev == dev && idle(b)) {
                held -= b.bytes;
                drop.push_back(b.ptr);
                if (b.done) (void)hipEventDestroy(b.done);
                g_bufs.erase(g_bufs.begin() + k);
            } else {
                ++k;
            }
        }
    }
    for (void *p : drop) (void)hipFree(p);
    Buf b;
    b.bytes = want;
    b.dev = dev;
    b.busy = true;
    if ((e = hipMalloc(&b.ptr, (size_t)want)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MOA_ERR_NOMEM, "scratch of %lld bytes: %s", (long long)want, hipGetErrorString(e));
    }
    if ((e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming)) != hipSuccess) {
        (void)hipFree(b.ptr);
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_bufs.push_back(b);
    }
    *ptr = b.ptr;
    return MOA_OK;
}

void scratch_free(void *ptr, hipStream_t stream) {
    if (!ptr) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (Buf &b : g_bufs) {
            if (b.ptr != ptr) continue;
            (void)hipEventRecord(b.done, stream);
            b.last = stream;
            b.used = true;
            b.busy = false;
            return;
        }
    }
    (void)hipFreeAsync(ptr, stream);   // allocated during stream capture
}

}  // namespace moa
