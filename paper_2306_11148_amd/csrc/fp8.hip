// Power-of-two scaled FP8 path. Eq. 3 is invariant under C = D_r^-1 ((D_r A)
// (B D_c)) D_c^-1 for diagonal D_r = diag(2^e_i), D_c = diag(2^f_j): the
// scales factor out of the k-sum, so they are applied exactly before rounding
// the operands to OCP E4M3 and removed exactly (ldexp) in the epilogue.
//
//   e_i = largest integer with amax_k |A[i,k]| * 2^e_i <= 448 (0 if the row
//         is zero); f_j likewise for column j of B.
//   qA[i,k] = RNE_e4m3(A[i,k] 2^e_i),  qB[k,j] = RNE_e4m3(B[k,j] 2^f_j)
//   C[i,j] = 2^-(e_i+f_j) sum_k qA[i,k] qB[k,j]          (one term)
// With the residual term r = x 2^e - q (exact in FP32) kept as
// l = RNE_e4m3(2^4 r):
//   C[i,j] = 2^-(e_i+f_j) (sum qA qB + 2^-4 (sum qA lB + sum lA qB))
// The factor 2^-4 is the E8M0 block scale of the residual operand of the
// scaled matrix-core step, so all three sums share one FP32 accumulator.
//
// Conditioning (HBM-bound): row exponents of A (one wave per row), column
// amax of B (atomic max on the bit patterns of |x|, which order like
// unsigned ints), then quantisation straight into record tiles (layout in
// ring_gemm.h): record (r, s) holds the 64 codes of k = 64s .. 64s+63 of row r
// of A, or of column r of B (B is transposed on the way). The two-term path
// keeps the residual codes in a second record array per operand. The
// contraction is the record-tile ring of ring_gemm.h with
// v_mfma_scale_f32_32x32x64_f8f6f4 steps.
#include "moa_internal.h"
#include "ring_gemm.h"
#include "tile_common.h"

namespace moa {
namespace {

using ring::GROUP;
using ring::padded_rows;
using ring::REC_BYTES;

constexpr int SLAB8 = 64;                // k per record: 64 E4M3 codes
static_assert(REC_BYTES == SLAB8, "one record holds one slab of codes");
// E8M0 block scales of the scaled matrix-core step: 2^(x - 127).
constexpr int kScaleOne = 0x7f;          // 2^0 (0 would mean 2^-127)
constexpr int kScaleLo = 0x7f - 4;       // 2^-4: residual codes carry a factor 2^4

typedef int i32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int pow2_exponent(float amax) {
    if (!(amax > 0.0f)) return 0;
    int E;
    const float f = frexpf(amax, &E);   // amax = f 2^E, f in [0.5, 1)
    // 448 = 0.875 * 2^9: f 2^(E+e) <= 0.875 2^9 decides e exactly.
    return (f <= 0.875f) ? 9 - E : 8 - E;
}

// Four values -> four E4M3 codes (round to nearest even), byte t = value t.
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

__device__ __forceinline__ float e4m3_value(uint32_t word, int byte) {
    switch (byte) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8((int)word, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8((int)word, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8((int)word, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8((int)word, 3);
    }
}

// hi and (2^4 x residual) codes of four scaled values.
__device__ __forceinline__ void quant4(const float v[4], bool two_term, uint32_t *hi, uint32_t *lo) {
    const uint32_t h = e4m3x4(v[0], v[1], v[2], v[3]);
    *hi = h;
    if (two_term) {
        float r[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = ldexpf(v[t] - e4m3_value(h, t), 4);
        *lo = e4m3x4(r[0], r[1], r[2], r[3]);
    }
}

__global__ void fill_u32_kernel(uint32_t *x, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) x[t] = 0u;
}

// One wave per row of A: e_i from amax |A[i, :]|.
__global__ __launch_bounds__(256) void row_exp_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                      int vec, int32_t *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    const float *row = A + i * n;
    float mx = 0.0f;
    if (vec) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll 8
        for (int64_t k = lane; k < n / 4; k += 64) {
            const float4 v = r4[k];
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
    } else {
        for (int64_t k = lane; k < n; k += 64) mx = fmaxf(mx, fabsf(row[k]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) e[i] = pow2_exponent(mx);
}

// Column amax of B: each thread takes one column over a band of 256 rows.
constexpr int COL_BAND = 256;
__global__ __launch_bounds__(256) void col_amax_kernel(const float *__restrict__ B, int64_t n,
                                                       int64_t p, uint32_t *__restrict__ amax) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.y * COL_BAND;
    if (j >= p) return;
    float mx = 0.0f;
    const int64_t k1 = min(n, k0 + COL_BAND);
#pragma unroll 16
    for (int64_t k = k0; k < k1; ++k) mx = fmaxf(mx, fabsf(B[k * p + j]));
    atomicMax(&amax[j], __float_as_uint(mx));
}

// --------------------------------------------------- record conditioning --

// Rows of A -> records. Chunk q = 16 codes of one record (4 per record);
// consecutive threads fill one KiB record tile contiguously.
template <bool TWO>
__global__ __launch_bounds__(256) void pack_rows_fp8_kernel(const float *__restrict__ A, int64_t m,
                                                            int64_t n, int64_t S, int vec,
                                                            const int32_t *__restrict__ e,
                                                            uint8_t *__restrict__ qa,
                                                            uint8_t *__restrict__ la) {
    const int64_t chunks = padded_rows(m) * S * 4;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256) {
        const int c = (int)(q & 3);
        const int64_t rr = (q >> 2) % GROUP;
        const int64_t gs = (q >> 2) / GROUP;
        const int64_t s = gs % S, g = gs / S;
        const int64_t r = g * GROUP + rr;
        const int64_t k = s * SLAB8 + c * 16;
        float x[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = 0.0f;
        if (r < m) {
            const float *src = A + r * n + k;
            if (vec && k + 16 <= n) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 v = reinterpret_cast<const float4 *>(src)[u];
                    x[4 * u] = v.x; x[4 * u + 1] = v.y; x[4 * u + 2] = v.z; x[4 * u + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if (k + t < n) x[t] = src[t];
            }
            const int er = e[r];
#pragma unroll
            for (int t = 0; t < 16; ++t) x[t] = ldexpf(x[t], er);
        }
        uint32_t hi[4], lo[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 4; ++u) quant4(x + 4 * u, TWO, &hi[u], &lo[u]);
        const int64_t at = ring::rec_byte(r, s, S) + c * 16;
        *reinterpret_cast<uint4 *>(qa + at) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        if (TWO) *reinterpret_cast<uint4 *>(la + at) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    }
}

// Columns of B -> records (transposed), 64 columns x one slab (64 k) per
// workgroup step. Thread t reads rows 4(t/16) .. +3 of columns 4(t%16) .. +3
// (each row of the block is 256 contiguous bytes), quantises them, turns the
// 4 x 4 codes around in registers and stores one dword per column into an LDS
// tile (row stride 17 dwords: the 64 lanes of a store hit 64 distinct banks).
// Then thread t writes bytes 16(t%4) .. +15 of the record of column t/4, so a
// wave stores one whole KiB record tile. Column exponents come from the column
// amax; workgroups with blockIdx.y == 0 also store them. Columns past p get
// zero records.
constexpr int TSTRIDE = 17;

__device__ __forceinline__ uint32_t byte_column(const uint32_t w[4], int c) {
    const int sh = 8 * c;
    return ((w[0] >> sh) & 0xFFu) | (((w[1] >> sh) & 0xFFu) << 8) | (((w[2] >> sh) & 0xFFu) << 16) |
           (((w[3] >> sh) & 0xFFu) << 24);
}

template <bool TWO>
__global__ __launch_bounds__(256) void pack_cols_fp8_kernel(const float *__restrict__ B, int64_t n,
                                                            int64_t p, int64_t S, int vec,
                                                            const uint32_t *__restrict__ amax,
                                                            int32_t *__restrict__ f_out,
                                                            uint8_t *__restrict__ qb,
                                                            uint8_t *__restrict__ lb) {
    __shared__ uint32_t tq[64 * TSTRIDE];
    __shared__ uint32_t tl[TWO ? 64 * TSTRIDE : 1];
    const int t = threadIdx.x;
    const int cg = t & 15, kq = t >> 4;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int64_t j = j0 + 4 * cg;                 // this thread's first column
    int fcol[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fcol[u] = (j + u < p) ? pow2_exponent(__uint_as_float(amax[j + u])) : 0;
        if (blockIdx.y == 0 && kq == 0 && j + u < p) f_out[j + u] = fcol[u];
    }
    const int jj = t >> 2, c = t & 3;              // writer: column j0 + jj, chunk c
    const bool writes = j0 + jj < padded_rows(p);
    for (int64_t s = blockIdx.y; s < S; s += gridDim.y) {
        uint32_t wq[4], wl[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t k = s * SLAB8 + 4 * kq + i;
            float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (k < n) {
                const float *row = B + k * p + j;
                if (vec && j + 4 <= p) {
                    const float4 x = *reinterpret_cast<const float4 *>(row);
                    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (j + u < p) v[u] = row[u];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = ldexpf(v[u], fcol[u]);
            quant4(v, TWO, &wq[i], &wl[i]);
        }
        __syncthreads();                           // the previous step's reads of the tiles are done
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            tq[(4 * cg + u) * TSTRIDE + kq] = byte_column(wq, u);
            if (TWO) tl[(4 * cg + u) * TSTRIDE + kq] = byte_column(wl, u);
        }
        __syncthreads();
        if (writes) {
            const uint32_t *r = tq + jj * TSTRIDE + 4 * c;
            const int64_t at = ring::rec_byte(j0 + jj, s, S) + 16 * c;
            *reinterpret_cast<uint4 *>(qb + at) = make_uint4(r[0], r[1], r[2], r[3]);
            if (TWO) {
                const uint32_t *q = tl + jj * TSTRIDE + 4 * c;
                *reinterpret_cast<uint4 *>(lb + at) = make_uint4(q[0], q[1], q[2], q[3]);
            }
        }
    }
}

// ------------------------------------------- row-major codes (exposed API) --

// qA (row-major, like A): 4 consecutive elements per thread.
__global__ __launch_bounds__(256) void quant_rows_kernel(const float *__restrict__ A, int64_t m,
                                                         int64_t n, const int32_t *__restrict__ e,
                                                         int two_term, uint8_t *__restrict__ q,
                                                         uint8_t *__restrict__ l) {
    const int64_t i = blockIdx.x;
    const int64_t k = ((int64_t)blockIdx.y * 256 + threadIdx.x) * 4;
    if (k >= n) return;
    const int ei = e[i];
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (k + t < n) ? ldexpf(A[i * n + k + t], ei) : 0.0f;
    uint32_t hi, lo = 0;
    quant4(v, two_term != 0, &hi, &lo);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (k + t < n) {
            q[i * n + k + t] = (uint8_t)(hi >> (8 * t));
            if (two_term) l[i * n + k + t] = (uint8_t)(lo >> (8 * t));
        }
}

// qB (row-major, like B): 4 consecutive columns x 4 rows per thread.
__global__ __launch_bounds__(256) void quant_cols_kernel(const float *__restrict__ B, int64_t n,
                                                         int64_t p, const uint32_t *__restrict__ amax,
                                                         int two_term, int32_t *__restrict__ f_out,
                                                         uint8_t *__restrict__ q,
                                                         uint8_t *__restrict__ l) {
    const int64_t k0 = (int64_t)blockIdx.y * 64, jb = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 15;      // 4 columns each
    const int ty = threadIdx.x >> 4;      // 16 rows, 4 passes
    const int64_t j = jb + tx * 4;
    int f[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f[t] = (j + t < p) ? pow2_exponent(__uint_as_float(amax[j + t])) : 0;
        if (blockIdx.y == 0 && ty == 0 && j + t < p) f_out[j + t] = f[t];
    }
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int64_t k = k0 + ty + 16 * pass;
        if (k >= n) continue;
        float v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (j + t < p) ? ldexpf(B[k * p + j + t], f[t]) : 0.0f;
        uint32_t hi, lo = 0;
        quant4(v, two_term != 0, &hi, &lo);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (j + t < p) {
                q[k * p + j + t] = (uint8_t)(hi >> (8 * t));
                if (two_term) l[k * p + j + t] = (uint8_t)(lo >> (8 * t));
            }
    }
}

// ---------------------------------------------------------- contraction --

// Fragments of 32 records x 32 codes: lane l reads row base + l%32, logical
// chunks 2(l/32) and 2(l/32) + 1 (k = 32(l/32) .. +31 of the slab); A and B
// use the same k assignment, which is all the step's dot product needs.
template <bool TWO> struct Fp8Mode {
    static constexpr bool SCALED = true;
    template <int FM, int FN> struct Frags {
        i32x8_t ah[FM], bh[FN], al[TWO ? FM : 1], bl[TWO ? FN : 1];
    };

    static __device__ __forceinline__ i32x8_t frag(const uint8_t *buf, int row, int half) {
        const i32x4_t x = ring::lds_chunk<i32x4_t>(buf, row, 2 * half);
        const i32x4_t y = ring::lds_chunk<i32x4_t>(buf, row, 2 * half + 1);
        return __builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, 6, 7);
    }

    // LDS rows: [A hi (BM)][A lo (BM)][B hi (BN)][B lo (BN)] (lo: two-term only)
    template <int BM, int BN, int FM, int FN>
    static __device__ __forceinline__ void read(const uint8_t *buf, int a_row, int b_row, int half,
                                                Frags<FM, FN> &f) {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            f.ah[a] = frag(buf, a_row + a * 32, half);
            if constexpr (TWO) f.al[a] = frag(buf, a_row + BM + a * 32, half);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            f.bh[b] = frag(buf, b_row + b * 32, half);
            if constexpr (TWO) f.bl[b] = frag(buf, b_row + BN + b * 32, half);
        }
    }

    // every element sees, per slab in ascending order: 2^-4 lA.qB, 2^-4 qA.lB
    // (two-term only), then qA.qB
    template <int FM, int FN>
    static __device__ __forceinline__ void mma(const Frags<FM, FN> &f, f32x16_t (&acc)[FM][FN]) {
        if constexpr (TWO) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        f.al[a], f.bh[b], acc[a][b], 0, 0, 0, kScaleLo, 0, kScaleOne);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        f.ah[a], f.bl[b], acc[a][b], 0, 0, 0, kScaleOne, 0, kScaleLo);
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    f.ah[a], f.bh[b], acc[a][b], 0, 0, 0, kScaleOne, 0, kScaleOne);
    }
};

struct Fp8Shape { int bm, bn, wm, wn, stages; };
constexpr Fp8Shape kOne[] = {{128, 128, 64, 64, 3}, {256, 256, 128, 64, 3}, {256, 256, 128, 64, 4},
                             {256, 256, 128, 64, 5}};
// Deeper rings pay off here: a slab carries 64 k, so a step is short next
// to the latency of its loads.
constexpr Fp8Shape kTwo[] = {{128, 128, 64, 64, 3}, {128, 128, 64, 32, 3}, {128, 128, 64, 32, 5},
                             {128, 128, 64, 32, 4}};
constexpr int kOneCount = sizeof(kOne) / sizeof(kOne[0]);
constexpr int kTwoCount = sizeof(kTwo) / sizeof(kTwo[0]);

template <int BM, int BN, int WM, int WN, bool TWO, int NST = ring::NSTAGE>
hipError_t launch_shape(const ring::Operands &op, hipStream_t st) {
    constexpr int NREC = TWO ? 2 : 1;
    const int tiles_m = (int)((op.m + BM - 1) / BM);
    const int tiles_n = (int)((op.p + BN - 1) / BN);
    hipLaunchKernelGGL((ring::single_kernel<BM, BN, WM, WN, NREC, Fp8Mode<TWO>, NST>), dim3(tiles_m * tiles_n),
                       dim3(ring::Cfg<BM, BN, WM, WN, NREC, NST>::THREADS), 0, st, op, tiles_m, tiles_n);
    return hipGetLastError();
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Fp8Workspace {
    uint32_t *amaxB;
    int32_t *e, *f;
    uint8_t *qA, *lA, *qB, *lB;
};

Fp8Workspace carve(void *ws, int64_t m, int64_t n, int64_t p, bool two) {
    const int64_t S = (n + SLAB8 - 1) / SLAB8;
    char *c = static_cast<char *>(ws);
    Fp8Workspace w;
    w.amaxB = reinterpret_cast<uint32_t *>(c); c += align256(4 * p);
    w.e = reinterpret_cast<int32_t *>(c); c += align256(4 * m);
    w.f = reinterpret_cast<int32_t *>(c); c += align256(4 * p);
    w.qA = reinterpret_cast<uint8_t *>(c); c += align256(ring::array_bytes(m, S));
    w.qB = reinterpret_cast<uint8_t *>(c); c += align256(ring::array_bytes(p, S));
    w.lA = two ? reinterpret_cast<uint8_t *>(c) : nullptr; c += two ? align256(ring::array_bytes(m, S)) : 0;
    w.lB = two ? reinterpret_cast<uint8_t *>(c) : nullptr;
    return w;
}

// Exponents of A's rows and amax of B's columns (shared by both layouts).
void scales(const float *A, int64_t m, int64_t n, const float *B, int64_t p, int32_t *e, uint32_t *amaxB,
            hipStream_t st) {
    if (p > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, amaxB, p);
    const int vec = (n % 4 == 0) && ((uintptr_t)A % 16 == 0);
    if (m > 0) hipLaunchKernelGGL(row_exp_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, A, m, n, vec, e);
    if (p > 0 && n > 0)
        hipLaunchKernelGGL(col_amax_kernel, dim3((unsigned)((p + 255) / 256), (unsigned)((n + COL_BAND - 1) / COL_BAND)),
                           dim3(256), 0, st, B, n, p, amaxB);
}

hipError_t pack_records(const moa_gemm_desc &d, bool two, const Fp8Workspace &w, hipStream_t st) {
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    const int64_t S = (d.n + SLAB8 - 1) / SLAB8;
    scales(A, d.m, d.n, B, d.p, w.e, w.amaxB, st);
    if (d.m > 0 && S > 0) {
        const int vec = (d.n % 4 == 0) && ((uintptr_t)A % 16 == 0);
        int64_t blocks = (padded_rows(d.m) * S * 4 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (two)
            hipLaunchKernelGGL(pack_rows_fp8_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, A, d.m, d.n, S,
                               vec, w.e, w.qA, w.lA);
        else
            hipLaunchKernelGGL(pack_rows_fp8_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, A, d.m, d.n, S,
                               vec, w.e, w.qA, w.lA);
    }
    if (d.p > 0) {   // also when S == 0: the epilogue reads the column exponents
        const int vec = (d.p % 4 == 0) && ((uintptr_t)B % 16 == 0);
        const dim3 grid((unsigned)((d.p + 63) / 64), (unsigned)(S < 1 ? 1 : S > 65535 ? 65535 : S));
        if (two)
            hipLaunchKernelGGL(pack_cols_fp8_kernel<true>, grid, dim3(256), 0, st, B, d.n, d.p, S, vec, w.amaxB,
                               w.f, w.qB, w.lB);
        else
            hipLaunchKernelGGL(pack_cols_fp8_kernel<false>, grid, dim3(256), 0, st, B, d.n, d.p, S, vec, w.amaxB,
                               w.f, w.qB, w.lB);
    }
    return hipGetLastError();
}

}  // namespace

int fp8_variant_count(bool two) { return two ? kTwoCount : kOneCount; }

void fp8_shape(bool two, int v, Plan *p) {
    const Fp8Shape s = two ? kTwo[v] : kOne[v];
    p->variant = v;
    p->tile_m = s.bm;
    p->tile_n = s.bn;
    p->tile_k = SLAB8;
    p->wave_m = s.wm;
    p->wave_n = s.wn;
    p->lane_m = p->lane_n = 0;
    p->threads = (s.bm / s.wm) * (s.bn / s.wn) * 64;
    p->lds_bytes = s.stages * (two ? 2 : 1) * (s.bm + s.bn) * REC_BYTES;
}

int64_t fp8_workspace_bytes(int64_t m, int64_t n, int64_t p, bool two) {
    const int64_t S = (n + SLAB8 - 1) / SLAB8;
    const int64_t rec = align256(ring::array_bytes(m, S)) + align256(ring::array_bytes(p, S));
    return align256(4 * p) * 2 + align256(4 * m) + (two ? 2 : 1) * rec;
}

hipError_t launch_fp8(const moa_gemm_desc &d, const Plan &plan, void *ws, hipStream_t st) {
    const bool two = (d.flags & MOA_FLAG_FP8_TWO_TERM) != 0;
    const Fp8Workspace w = carve(ws, d.m, d.n, d.p, two);
    hipError_t err;
    {
        TraceScope ts(MOA_K_FP8_QUANT, st);
        err = pack_records(d, two, w, st);
    }
    if (err != hipSuccess) return err;
    TraceScope ts(two ? MOA_K_FP8_2TERM : MOA_K_FP8, st);
    ring::Operands op;
    op.a0 = w.qA; op.a1 = w.lA;
    op.b0 = w.qB; op.b1 = w.lB;
    op.C = static_cast<float *>(d.C);
    op.row_exp = w.e;
    op.col_exp = w.f;
    op.m = d.m; op.p = d.p;
    op.S = (d.n + SLAB8 - 1) / SLAB8;
    op.accumulate = d.accumulate;
    if (two) {
        switch (plan.variant) {
        case 0: return launch_shape<128, 128, 64, 64, true>(op, st);
        case 1: return launch_shape<128, 128, 64, 32, true>(op, st);
        case 2: return launch_shape<128, 128, 64, 32, true, 5>(op, st);
        default: return launch_shape<128, 128, 64, 32, true, 4>(op, st);
        }
    }
    switch (plan.variant) {
    case 0: return launch_shape<128, 128, 64, 64, false>(op, st);
    case 1: return launch_shape<256, 256, 128, 64, false>(op, st);
    case 2: return launch_shape<256, 256, 128, 64, false, 4>(op, st);
    default: return launch_shape<256, 256, 128, 64, false, 5>(op, st);
    }
}

hipError_t launch_quantise_fp8(const float *A, int64_t m, int64_t n, const float *B, int64_t p,
                               bool two, int32_t *e, uint8_t *qA, uint8_t *lA, int32_t *f,
                               uint8_t *qB, uint8_t *lB, uint32_t *amax, hipStream_t st) {
    uint32_t *amaxB = amax + m;
    scales(A, m, n, B, p, e, amaxB, st);
    if (m > 0 && n > 0)
        hipLaunchKernelGGL(quant_rows_kernel, dim3((unsigned)m, (unsigned)((n + 1023) / 1024)), dim3(256), 0, st, A,
                           m, n, e, (int)two, qA, lA);
    if (p > 0)
        hipLaunchKernelGGL(quant_cols_kernel, dim3((unsigned)((p + 63) / 64), (unsigned)((n + 63) / 64 > 0 ? (n + 63) / 64 : 1)),
                           dim3(256), 0, st, B, n, p, amaxB, (int)two, f, qB, lB);
    return hipGetLastError();
}

}  // namespace moa
