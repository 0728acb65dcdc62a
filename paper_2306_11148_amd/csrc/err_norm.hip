// Normwise error of a result X against an FP64 reference R, in FP64:
//   out[0] = sum_t (X[t] - R[t])^2,  out[1] = sum_t R[t]^2.
// Two stages with a fixed grid and fixed reduction trees, so the sums (and
// the reported error) do not change from run to run.
#include "moa_internal.h"

namespace moa {
namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void err_partial_kernel(const T *__restrict__ X,
                                                               const double *__restrict__ R,
                                                               int64_t count,
                                                               double *__restrict__ partials) {
    __shared__ double s_num[kThreads], s_den[kThreads];
    double num = 0.0, den = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count; t += stride) {
        const double r = R[t];
        const double d = (double)X[t] - r;
        num = __builtin_fma(d, d, num);
        den = __builtin_fma(r, r, den);
    }
    s_num[threadIdx.x] = num;
    s_den[threadIdx.x] = den;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_num[threadIdx.x] += s_num[threadIdx.x + w];
            s_den[threadIdx.x] += s_den[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s_num[0];
        partials[2 * blockIdx.x + 1] = s_den[0];
    }
}

__global__ __launch_bounds__(kThreads) void err_final_kernel(const double *__restrict__ partials,
                                                             int nblocks, double *__restrict__ out) {
    __shared__ double s_num[kThreads], s_den[kThreads];
    double num = 0.0, den = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        num += partials[2 * b];
        den += partials[2 * b + 1];
    }
    s_num[threadIdx.x] = num;
    s_den[threadIdx.x] = den;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_num[threadIdx.x] += s_num[threadIdx.x + w];
            s_den[threadIdx.x] += s_den[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_num[0];
        out[1] = s_den[0];
    }
}

}  // namespace

hipError_t launch_error_norm(int64_t count, moa_dtype xt, const void *X, const double *R,
                             double *out, double *partials, int nblocks, hipStream_t st) {
    if (xt == MOA_F64)
        hipLaunchKernelGGL(err_partial_kernel<double>, dim3(nblocks), dim3(kThreads), 0, st,
                           static_cast<const double *>(X), R, count, partials);
    else
        hipLaunchKernelGGL(err_partial_kernel<float>, dim3(nblocks), dim3(kThreads), 0, st,
                           static_cast<const float *>(X), R, count, partials);
    hipLaunchKernelGGL(err_final_kernel, dim3(1), dim3(kThreads), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace moa
