// The ipophp family (conclusion and appendix: one formulation for the
// Hadamard product, the Kronecker product and the matrix product; higher
// dimensional contractions as many parallel 2-d products).
//
//   Hadamard:  C[i,j] := A[i,j] B[i,j]                          (m x n)
//   Kronecker: C[i p + k, j q + l] := A[i,j] B[k,l]             A m x n, B p x q
//   batched:   C[b] := A[b] B[b]                                (grouped launch)
//
// Every element of the first two is one product (plus, in the accumulate
// form, one addition to C), each rounded to the element type: floating-point
// contraction is off in these kernels, so results are bitwise those of the
// definition. Both are bound by HBM traffic: the Kronecker kernel writes C
// row by row (row i p + k of C is A[i, :] (x) B[k, :]), A and B stay in cache.
#include <algorithm>
#include <vector>

#include "moa_internal.h"

namespace moa {
namespace {

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int N = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int N = 2; };

template <typename T>
__device__ __forceinline__ T product(T a, T b, const T *c, int accumulate) {
#pragma clang fp contract(off)
    T v = a * b;
    if (accumulate) v = v + *c;
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void hadamard_kernel(const T *A, const T *B, T *C, int64_t count, int vec,
                                                       int accumulate) {   // C may be A or B (in place)
    using V = typename Vec16<T>::type;
    constexpr int N = Vec16<T>::N;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nvec = vec ? count / N : 0;
    for (int64_t t = t0; t < nvec; t += stride) {
        const V a = reinterpret_cast<const V *>(A)[t];
        const V b = reinterpret_cast<const V *>(B)[t];
        V c = accumulate ? reinterpret_cast<V *>(C)[t] : V{};   // C is read only when accumulating
        const T *pa = reinterpret_cast<const T *>(&a);
        const T *pb = reinterpret_cast<const T *>(&b);
        T *pc = reinterpret_cast<T *>(&c);
#pragma unroll
        for (int e = 0; e < N; ++e) pc[e] = product(pa[e], pb[e], pc + e, accumulate);
        reinterpret_cast<V *>(C)[t] = c;
    }
    for (int64_t x = nvec * N + t0; x < count; x += stride) C[x] = product(A[x], B[x], C + x, accumulate);
}

// Thread t owns columns c0 .. c0 + N - 1 of C (j = c / q, l = c mod q, found
// once in 32-bit arithmetic: the entry point keeps n q below 2^31) and walks
// rows r = i p + k of C; row r is A[i, :] (x) B[k, :].
template <typename T>
__global__ __launch_bounds__(256) void kronecker_kernel(const T *__restrict__ A, const T *__restrict__ B,
                                                        T *__restrict__ C, int64_t m, int64_t n, int64_t p,
                                                        int64_t q, int vec, int accumulate) {
    using V = typename Vec16<T>::type;
    constexpr int N = Vec16<T>::N;
    const int64_t rows = m * p;
    const int cols = (int)(n * q), qq = (int)q;
    for (int64_t c0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * N; c0 < cols;
         c0 += (int64_t)gridDim.x * 256 * N) {
        int jj[N], ll[N];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const int c = (int)min(c0 + e, (int64_t)cols - 1);
            jj[e] = c / qq;
            ll[e] = c - jj[e] * qq;
        }
        const bool full = vec && c0 + N <= cols;
        for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
            const int64_t i = r / p, k = r - i * p;
            const T *arow = A + i * n;
            const T *brow = B + k * q;
            T *crow = C + r * (int64_t)cols;
            if (full) {
                V out = accumulate ? *reinterpret_cast<const V *>(crow + c0) : V{};
                T *po = reinterpret_cast<T *>(&out);
#pragma unroll
                for (int e = 0; e < N; ++e) po[e] = product(arow[jj[e]], brow[ll[e]], po + e, accumulate);
                *reinterpret_cast<V *>(crow + c0) = out;
            } else {
                for (int e = 0; e < N && c0 + e < cols; ++e)
                    crow[c0 + e] = product(arow[jj[e]], brow[ll[e]], crow + c0 + e, accumulate);
            }
        }
    }
}

}  // namespace

hipError_t launch_hadamard(int64_t count, moa_dtype dt, const void *A, const void *B, void *C, int accumulate,
                           hipStream_t st) {
    int64_t blocks = (count + 1023) / 1024;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 8 * kNumCUs));
    const bool aligned = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && ((uintptr_t)C % 16 == 0);
    TraceScope ts(MOA_K_HADAMARD, st);
    if (dt == MOA_F64)
        hipLaunchKernelGGL(hadamard_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                           static_cast<const double *>(A), static_cast<const double *>(B), static_cast<double *>(C),
                           count, (int)aligned, accumulate);
    else
        hipLaunchKernelGGL(hadamard_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                           static_cast<const float *>(A), static_cast<const float *>(B), static_cast<float *>(C),
                           count, (int)aligned, accumulate);
    return hipGetLastError();
}

hipError_t launch_kronecker(int64_t m, int64_t n, int64_t p, int64_t q, moa_dtype dt, const void *A, const void *B,
                            void *C, int accumulate, hipStream_t st) {
    const int64_t cols = n * q, rows = m * p;
    const int N = dt == MOA_F64 ? 2 : 4;
    const bool vec = (cols % N == 0) && ((uintptr_t)C % 16 == 0);
    // about 2048 workgroups: all column chunks of a row, rows shared out
    const int64_t gx = std::min<int64_t>((cols + 256 * N - 1) / (256 * N), 64);
    const dim3 grid((unsigned)gx, (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 2048 / gx)));
    TraceScope ts(MOA_K_KRONECKER, st);
    if (dt == MOA_F64)
        hipLaunchKernelGGL(kronecker_kernel<double>, grid, dim3(256), 0, st, static_cast<const double *>(A),
                           static_cast<const double *>(B), static_cast<double *>(C), m, n, p, q, (int)vec,
                           accumulate);
    else
        hipLaunchKernelGGL(kronecker_kernel<float>, grid, dim3(256), 0, st, static_cast<const float *>(A),
                           static_cast<const float *>(B), static_cast<float *>(C), m, n, p, q, (int)vec,
                           accumulate);
    return hipGetLastError();
}

}  // namespace moa

using namespace moa;

namespace {
bool spans_overlap(const void *x, int64_t xb, const void *y, int64_t yb) {
    if (xb == 0 || yb == 0) return false;
    const uintptr_t x0 = (uintptr_t)x, y0 = (uintptr_t)y;
    return x0 < y0 + (uintptr_t)yb && y0 < x0 + (uintptr_t)xb;
}
}  // namespace

extern "C" {

moa_status moa_hadamard(int64_t m, int64_t n, int32_t dtype, const void *A, const void *B, void *C,
                        int32_t accumulate, void *stream) {
    try {
        if (m < 0 || n < 0) return fail(MOA_ERR_SHAPE, "negative shape");
        if (dtype != MOA_F64 && dtype != MOA_F32) return fail(MOA_ERR_INVALID, "unknown dtype %d", dtype);
        const int64_t es = dtype == MOA_F64 ? 8 : 4;
        int64_t count = 0;
        if (__builtin_mul_overflow(m, n, &count) || count > INT64_MAX / es) return fail(MOA_ERR_SHAPE, "size overflow");
        if (count == 0) return MOA_OK;
        if (!A || !B || !C) return fail(MOA_ERR_INVALID, "null pointer");
        if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) % (uintptr_t)es)
            return fail(MOA_ERR_INVALID, "pointers must be aligned to the element size");
        // C may be A or B exactly (elementwise), but not a shifted overlap
        if ((C != A && spans_overlap(C, count * es, A, count * es)) ||
            (C != B && spans_overlap(C, count * es, B, count * es)))
            return fail(MOA_ERR_INVALID, "C partially overlaps A or B");
        const hipError_t e = launch_hadamard(count, (moa_dtype)dtype, A, B, C, accumulate != 0,
                                             static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "hadamard launch");
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_kronecker(int64_t m, int64_t n, int64_t p, int64_t q, int32_t dtype, const void *A, const void *B,
                         void *C, int32_t accumulate, void *stream) {
    try {
        if (m < 0 || n < 0 || p < 0 || q < 0) return fail(MOA_ERR_SHAPE, "negative shape");
        if (dtype != MOA_F64 && dtype != MOA_F32) return fail(MOA_ERR_INVALID, "unknown dtype %d", dtype);
        const int64_t es = dtype == MOA_F64 ? 8 : 4;
        int64_t rows, cols, count, na, nb;
        if (__builtin_mul_overflow(m, p, &rows) || __builtin_mul_overflow(n, q, &cols) ||
            __builtin_mul_overflow(rows, cols, &count) || count > INT64_MAX / es ||
            __builtin_mul_overflow(m, n, &na) || __builtin_mul_overflow(p, q, &nb))
            return fail(MOA_ERR_SHAPE, "size overflow");
        if (cols > INT32_MAX) return fail(MOA_ERR_SHAPE, "n q = %lld exceeds 2^31 - 1", (long long)cols);
        if (count == 0) return MOA_OK;
        if (!A || !B || !C) return fail(MOA_ERR_INVALID, "null pointer");
        if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) % (uintptr_t)es)
            return fail(MOA_ERR_INVALID, "pointers must be aligned to the element size");
        if (spans_overlap(C, count * es, A, na * es) || spans_overlap(C, count * es, B, nb * es))
            return fail(MOA_ERR_INVALID, "C overlaps A or B");
        const hipError_t e = launch_kronecker(m, n, p, q, (moa_dtype)dtype, A, B, C, accumulate != 0,
                                              static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "kronecker launch");
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_gemm_batched(const moa_gemm_desc *first, int64_t batch, int64_t stride_a, int64_t stride_b,
                            int64_t stride_c, void *stream) {
    try {
        if (!first) return fail(MOA_ERR_INVALID, "null descriptor");
        if (batch < 0 || stride_a < 0 || stride_b < 0 || stride_c < 0)
            return fail(MOA_ERR_INVALID, "negative batch or stride");
        if (batch == 0) return MOA_OK;
        const int64_t es = first->dtype == MOA_F64 ? 8 : 4;
        std::vector<moa_gemm_desc> descs((size_t)batch, *first);
        for (int64_t b = 0; b < batch; ++b) {
            int64_t oa, ob, oc;
            if (__builtin_mul_overflow(b, stride_a * es, &oa) || __builtin_mul_overflow(b, stride_b * es, &ob) ||
                __builtin_mul_overflow(b, stride_c * es, &oc))
                return fail(MOA_ERR_SHAPE, "batch offset overflow");
            if (first->A) descs[b].A = static_cast<const char *>(first->A) + oa;
            if (first->B) descs[b].B = static_cast<const char *>(first->B) + ob;
            if (first->C) descs[b].C = static_cast<char *>(first->C) + oc;
        }
        return moa_gemm_grouped(descs.data(), batch, stream);
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

}  // extern "C"
