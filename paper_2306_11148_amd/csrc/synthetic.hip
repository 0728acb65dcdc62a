// Synthetic operands drawn on the device (the serving workload's requests are
// (shape, path, seed); their operands are generated where they are used).
//
// Generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011): per round the
// counter words c0 and c2 are multiplied by 0xD2511F53 and 0xCD9E8D57 into
// 64-bit products, and the new counter is (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1),
// hi(c0 M0) ^ c3 ^ k1, lo(c0 M0)); the key is bumped by (0x9E3779B9,
// 0xBB67AE85) between rounds, everything modulo 2^32.
//
// Element e (row-major flat index) of operand `tag` of a request with 64-bit
// `seed`: pair q = e / 2 draws one block with counter (q mod 2^32, q / 2^32,
// tag, 0) and key (seed mod 2^32, seed / 2^32); element 2q takes words x0, x1
// and element 2q + 1 words x2, x3. With S the sum of the four 16-bit halves
// of its two words, the value is the FP32 product (2 S - 4 * 65535) * c with
// c the FP32 value nearest sqrt(3) * 2^-17 (a centred sum of four uniform
// variates, unit variance). The integer has at most 19 bits, so its
// conversion is exact and the product is the only rounding.
//
// One thread per pair; 8-byte stores when the array is 8-byte aligned.
#include "moa_internal.h"

namespace moa {
namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr float kScale = 0x1.bb67aep-17f;   // nearest FP32 to sqrt(3) * 2^-17

__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c0;
        const uint64_t p1 = (uint64_t)kM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
}

__device__ __forceinline__ float value(uint32_t a, uint32_t b) {
    const int s = (int)(a & 0xFFFFu) + (int)(a >> 16) + (int)(b & 0xFFFFu) + (int)(b >> 16);
    return (float)(2 * s - 4 * 65535) * kScale;
}

__global__ __launch_bounds__(256) void synthetic_kernel(float *__restrict__ X, int64_t count, uint32_t k0,
                                                        uint32_t k1, uint32_t tag, int vec) {
    const int64_t pairs = (count + 1) / 2;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < pairs; q += stride) {
        uint32_t c0 = (uint32_t)q, c1 = (uint32_t)((uint64_t)q >> 32), c2 = tag, c3 = 0;
        philox10(c0, c1, c2, c3, k0, k1);
        const float v0 = value(c0, c1), v1 = value(c2, c3);
        const int64_t e = 2 * q;
        if (vec && e + 1 < count) {
            *reinterpret_cast<float2 *>(X + e) = make_float2(v0, v1);
        } else {
            X[e] = v0;
            if (e + 1 < count) X[e + 1] = v1;
        }
    }
}

}  // namespace

hipError_t launch_synthetic(float *X, int64_t count, uint64_t seed, uint32_t tag, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int64_t pairs = (count + 1) / 2;
    int64_t blocks = (pairs + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    const int vec = ((uintptr_t)X % 8) == 0;
    hipLaunchKernelGGL(synthetic_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, count,
                       (uint32_t)seed, (uint32_t)(seed >> 32), tag, vec);
    return hipGetLastError();
}

}  // namespace moa

using namespace moa;

extern "C" moa_status moa_fill_synthetic(float *X, int64_t count, uint64_t seed, uint32_t operand, void *stream) {
    if (count < 0) return fail(MOA_ERR_SHAPE, "negative count");
    if (count == 0) return MOA_OK;
    if (!X) return fail(MOA_ERR_INVALID, "null pointer");
    if ((uintptr_t)X % 4) return fail(MOA_ERR_INVALID, "X must be aligned to 4 bytes");
    const hipError_t e = launch_synthetic(X, count, seed, operand, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "synthetic fill launch");
    return MOA_OK;
}
