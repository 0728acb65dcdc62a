// moa_gemm_noalloc: the product of moa_gemm with every scratch buffer (record
// tiles, exponents, split-k partials) placed in one fixed array of device
// memory that the library defines, so that a call allocates nothing.
//
// `scratch` is a file-scope device array: the code object loader gives each
// GPU its own copy, at its own address, when the library's kernels are first
// loaded there, and keeps it until the process ends. In host code the name
// `scratch` is only a host-side stand-in for that array and must never be
// passed to a kernel or a copy; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
#include <mutex>

#include "moa_internal.h"

namespace moa {
namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[MOA_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch`.
moa_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MOA_ERR_UNSUPPORTED, "device %d is beyond the %d devices the fixed scratch serves", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MOA_OK;
}

}  // namespace
}  // namespace moa

using namespace moa;

extern "C" moa_status moa_gemm_noalloc(const moa_gemm_desc *desc, void *stream) {
    try {
        if (!desc) return fail(MOA_ERR_INVALID, "null descriptor");
        moa_status s = validate(*desc, true);
        if (s != MOA_OK) return s;
        if (desc->m == 0 || desc->p == 0) return MOA_OK;
        void *ws = nullptr;
        if ((s = scratch_address(&ws)) != MOA_OK) return s;
        return run_gemm_in(*desc, static_cast<hipStream_t>(stream), ws, MOA_NOALLOC_SCRATCH_BYTES);
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}
