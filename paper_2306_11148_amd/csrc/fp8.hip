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
#include <algorithm>
#include <vector>

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

// One wave: e_i of row i of A from amax |A[i, :]| (all 64 lanes take part).
__device__ __forceinline__ void row_exp_wave(const float *__restrict__ A, int64_t i, int64_t n, int vec,
                                             int lane, int32_t *__restrict__ e) {
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

// One wave per row of A.
__global__ __launch_bounds__(256) void row_exp_kernel(const float *__restrict__ A, int64_t m, int64_t n,
                                                      int vec, int32_t *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i < m) row_exp_wave(A, i, n, vec, threadIdx.x & 63, e);
}

// Column amax of B: one thread per column over a band of COL_BAND rows.
constexpr int COL_BAND = 256;
__device__ __forceinline__ void col_amax_thread(const float *__restrict__ B, int64_t n, int64_t p, int64_t j,
                                                int64_t k0, uint32_t *__restrict__ amax) {
    float mx = 0.0f;
    const int64_t k1 = min(n, k0 + COL_BAND);
#pragma unroll 16
    for (int64_t k = k0; k < k1; ++k) mx = fmaxf(mx, fabsf(B[k * p + j]));
    atomicMax(&amax[j], __float_as_uint(mx));
}

__global__ __launch_bounds__(256) void col_amax_kernel(const float *__restrict__ B, int64_t n,
                                                       int64_t p, uint32_t *__restrict__ amax) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < p) col_amax_thread(B, n, p, j, (int64_t)blockIdx.y * COL_BAND, amax);
}

// --------------------------------------------------- record conditioning --

// Rows of A -> records. Chunk q = 16 codes of one record (4 per record);
// consecutive chunks fill one KiB record tile contiguously.
template <bool TWO>
__device__ __forceinline__ void pack_rows_fp8_chunk(const float *__restrict__ A, int64_t m, int64_t n,
                                                    int64_t S, int vec, const int32_t *__restrict__ e,
                                                    uint8_t *__restrict__ qa, uint8_t *__restrict__ la,
                                                    int64_t q) {
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

template <bool TWO>
__global__ __launch_bounds__(256) void pack_rows_fp8_kernel(const float *__restrict__ A, int64_t m,
                                                            int64_t n, int64_t S, int vec,
                                                            const int32_t *__restrict__ e,
                                                            uint8_t *__restrict__ qa,
                                                            uint8_t *__restrict__ la) {
    const int64_t chunks = padded_rows(m) * S * 4;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256)
        pack_rows_fp8_chunk<TWO>(A, m, n, S, vec, e, qa, la, q);
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

// Column exponents of the 64 columns of block bx (threads 0 .. 63).
__device__ __forceinline__ void write_col_exps(const uint32_t *__restrict__ amax, int64_t p, int64_t bx,
                                               int32_t *__restrict__ f_out) {
    const int64_t j = bx * 64 + threadIdx.x;
    if (threadIdx.x < 64 && j < p) f_out[j] = pow2_exponent(__uint_as_float(amax[j]));
}

// Block (bx, s): columns 64 bx .. 64 bx + 63, slab s < S. All 256 threads
// take part; the LDS tiles are free again when it returns.
template <bool TWO>
__device__ __forceinline__ void pack_cols_fp8_block(const float *__restrict__ B, int64_t n, int64_t p,
                                                    int64_t S, int vec, const uint32_t *__restrict__ amax,
                                                    uint8_t *__restrict__ qb, uint8_t *__restrict__ lb,
                                                    int64_t bx, int64_t s, uint32_t *tq, uint32_t *tl) {
    const int t = threadIdx.x;
    const int cg = t & 15, kq = t >> 4;
    const int64_t j0 = bx * 64;
    const int64_t j = j0 + 4 * cg;                 // this thread's first column
    int fcol[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) fcol[u] = (j + u < p) ? pow2_exponent(__uint_as_float(amax[j + u])) : 0;
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
    __syncthreads();                               // earlier readers of the tiles are done
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        tq[(4 * cg + u) * TSTRIDE + kq] = byte_column(wq, u);
        if (TWO) tl[(4 * cg + u) * TSTRIDE + kq] = byte_column(wl, u);
    }
    __syncthreads();
    const int jj = t >> 2, c = t & 3;              // writer: column j0 + jj, chunk c
    if (j0 + jj < padded_rows(p)) {
        const uint32_t *r = tq + jj * TSTRIDE + 4 * c;
        const int64_t at = ring::rec_byte(j0 + jj, s, S) + 16 * c;
        *reinterpret_cast<uint4 *>(qb + at) = make_uint4(r[0], r[1], r[2], r[3]);
        if (TWO) {
            const uint32_t *q = tl + jj * TSTRIDE + 4 * c;
            *reinterpret_cast<uint4 *>(lb + at) = make_uint4(q[0], q[1], q[2], q[3]);
        }
    }
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
    if (blockIdx.y == 0) write_col_exps(amax, p, blockIdx.x, f_out);
    for (int64_t s = blockIdx.y; s < S; s += gridDim.y)
        pack_cols_fp8_block<TWO>(B, n, p, S, vec, amax, qb, lb, blockIdx.x, s, tq, tl);
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

// ------------------------------------------------ grouped (persistent) --
// Independent FP8 products of one term count share one launch sequence:
// clear (claim counter + every member's column amax), scales (row exponents
// and column amax of every member), records (every member's rows and column
// blocks), contraction (persistent workgroups claim tiles of all members from
// one counter). The scale and record steps each walk one work list over all
// members, so large and small members share the machine evenly. Every element
// sees the operation sequence of the single-product path, so results are
// bitwise those of moa_gemm.
struct Fp8Member {
    ring::Operands op;                  // the contraction's view (read by ring::tile in place)
    const float *A, *B;
    uint8_t *qa, *la, *qb, *lb;         // record arrays (la, lb: two-term only)
    int32_t *e, *f;                     // row / column exponents
    uint32_t *amaxB;                    // column amax (bit patterns)
    int64_t m, n, p, S;
    int64_t first_tile;                 // first contraction work-list id
    int64_t scale_first;                // first scale work-list id
    int64_t pack_first;                 // first record work-list id
    int32_t tiles_n, reserved;
    int32_t row_items;                  // scale items: row_items (4 rows each), then
    int32_t col_amax_x;                 //   col_amax_x * ceil(n / COL_BAND) column bands
    int32_t pack_row_items;             // record items: pack_row_items (256 chunks each), then
    int32_t pack_col_x;                 //   pack_col_x * max(S, 1) 64-column blocks
    int32_t vec_a, vec_b;
};

template <int64_t Fp8Member::*F>
__device__ __forceinline__ int find_member(const Fp8Member *__restrict__ g, int count, int64_t item) {
    int lo = 0, hi = count - 1;         // last member whose list starts at or before item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g[mid].*F <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void grouped_scales_kernel(const Fp8Member *__restrict__ g, int count,
                                                             int64_t total) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int k = __builtin_amdgcn_readfirstlane(find_member<&Fp8Member::scale_first>(g, count, item));
        const Fp8Member &d = g[k];
        const int64_t local = item - d.scale_first;
        if (local < d.row_items) {
            const int64_t i = local * 4 + wave;
            if (i < d.m) row_exp_wave(d.A, i, d.n, d.vec_a, lane, d.e);
        } else {
            const int64_t b = local - d.row_items;
            const int64_t j = (b % d.col_amax_x) * 256 + threadIdx.x;
            if (j < d.p) col_amax_thread(d.B, d.n, d.p, j, (b / d.col_amax_x) * COL_BAND, d.amaxB);
        }
    }
}

template <bool TWO>
__global__ __launch_bounds__(256) void grouped_records_kernel(const Fp8Member *__restrict__ g, int count,
                                                              int64_t total) {
    __shared__ uint32_t tq[64 * TSTRIDE];
    __shared__ uint32_t tl[TWO ? 64 * TSTRIDE : 1];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int k = __builtin_amdgcn_readfirstlane(find_member<&Fp8Member::pack_first>(g, count, item));
        const Fp8Member &d = g[k];
        const int64_t local = item - d.pack_first;
        if (local < d.pack_row_items) {
            const int64_t q = local * 256 + threadIdx.x;
            if (q < padded_rows(d.m) * d.S * 4)
                pack_rows_fp8_chunk<TWO>(d.A, d.m, d.n, d.S, d.vec_a, d.e, d.qa, d.la, q);
        } else {
            const int64_t b = local - d.pack_row_items;
            const int64_t bx = b % d.pack_col_x, s = b / d.pack_col_x;
            if (s == 0) write_col_exps(d.amaxB, d.p, bx, d.f);
            if (s < d.S) pack_cols_fp8_block<TWO>(d.B, d.n, d.p, d.S, d.vec_b, d.amaxB, d.qb, d.lb, bx, s, tq, tl);
        }
    }
}

struct Fp8Shape { int bm, bn, wm, wn, stages; };
constexpr Fp8Shape kOne[] = {{128, 128, 64, 64, 3}, {256, 256, 128, 64, 3}, {256, 256, 128, 64, 4},
                             {256, 256, 128, 64, 5}};
// Deeper rings pay off here: a slab carries 64 k, so a step is short next
// to the latency of its loads.
// The rectangular two-term blocks (8 waves of 64 x 64, 144 KB ring) read a
// third less LDS per matrix-core step than 128 x 128 with 64 x 32 waves; a
// wave's 96 LDS rows may span two record arrays. 256 x 128 is the default
// for large products (8192 x 4096 x 8192: 0.75 vs 0.83-0.89 ms).
constexpr Fp8Shape kTwo[] = {{128, 128, 64, 64, 3}, {128, 128, 64, 32, 3}, {128, 128, 64, 32, 5},
                             {128, 128, 64, 32, 4}, {128, 256, 64, 64, 3}, {256, 128, 64, 64, 3}};
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

template <bool TWO, int BM, int BN, int WM, int WN, int NST>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void fp8_grouped_kernel(
    const Fp8Member *__restrict__ g, int count, int64_t total_tiles, unsigned long long *__restrict__ counter) {
    constexpr int NREC = TWO ? 2 : 1;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[ring::Cfg<BM, BN, WM, WN, NREC, NST>::LDS];
    __shared__ int64_t s_tile;
    for (;;) {
        __syncthreads();                // nobody still reads lds or s_tile
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= total_tiles) break;
        const int k = __builtin_amdgcn_readfirstlane(find_member<&Fp8Member::first_tile>(g, count, tile));
        const Fp8Member &d = g[k];
        const int64_t local = tile - d.first_tile;
        const int64_t tm = local / d.tiles_n, tn = local - tm * d.tiles_n;
        ring::tile<BM, BN, WM, WN, NREC, Fp8Mode<TWO>, NST>(d.op, __builtin_amdgcn_readfirstlane((int)tm) * (int64_t)BM,
                                                            __builtin_amdgcn_readfirstlane((int)tn) * (int64_t)BN, lds);
    }
}

// Block shapes of the persistent launch: two terms 128 x 128 with 8 waves and
// a 4-deep ring (128 KiB LDS, one workgroup per CU); one term 128 x 128 with
// 4 waves and a 3-deep ring (48 KiB; its registers allow two per CU -- asking
// the compiler for three makes it spill).
constexpr int G_BM = 128, G_BN = 128;
constexpr int G_PER_CU_TWO = 1, G_PER_CU_ONE = 2;

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Fp8Workspace {
    uint32_t *amaxA, *amaxB;
    int32_t *e, *f;
    uint8_t *qA, *lA, *qB, *lB;
};

Fp8Workspace carve(void *ws, int64_t m, int64_t n, int64_t p, bool two) {
    const int64_t S = (n + SLAB8 - 1) / SLAB8;
    char *c = static_cast<char *>(ws);
    Fp8Workspace w;
    w.amaxB = reinterpret_cast<uint32_t *>(c); c += align256(4 * p);
    w.amaxA = reinterpret_cast<uint32_t *>(c); c += align256(4 * m);
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

// Exponents and records of one operand. A "row operand" is consumed row by
// row (A's rows: exponents e); a "column operand" column by column (B's
// columns: exponents f). `X` is row-major; `by_rows` says whether the wanted
// vectors are its rows (X is rows x K) or its columns (X is K x rows).
void operand_records(const float *X, int64_t rows, int64_t K, int64_t S, bool by_rows, bool two, uint32_t *amax,
                     int32_t *exps, uint8_t *q, uint8_t *l, hipStream_t st) {
    if (rows == 0) return;
    if (by_rows) {
        const int vec = (K % 4 == 0) && ((uintptr_t)X % 16 == 0);
        hipLaunchKernelGGL(row_exp_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, X, rows, K, vec, exps);
        if (S > 0) {
            int64_t blocks = (padded_rows(rows) * S * 4 + 255) / 256;
            if (blocks > 65536) blocks = 65536;
            if (two)
                hipLaunchKernelGGL(pack_rows_fp8_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, K,
                                   S, vec, exps, q, l);
            else
                hipLaunchKernelGGL(pack_rows_fp8_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, K,
                                   S, vec, exps, q, l);
        }
        return;
    }
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, amax, rows);
    if (K > 0)
        hipLaunchKernelGGL(col_amax_kernel, dim3((unsigned)((rows + 255) / 256), (unsigned)((K + COL_BAND - 1) / COL_BAND)),
                           dim3(256), 0, st, X, K, rows, amax);
    // also when S == 0: the epilogue reads the exponents
    const int vec = (rows % 4 == 0) && ((uintptr_t)X % 16 == 0);
    const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)(S < 1 ? 1 : S > 65535 ? 65535 : S));
    if (two)
        hipLaunchKernelGGL(pack_cols_fp8_kernel<true>, grid, dim3(256), 0, st, X, K, rows, S, vec, amax, exps, q, l);
    else
        hipLaunchKernelGGL(pack_cols_fp8_kernel<false>, grid, dim3(256), 0, st, X, K, rows, S, vec, amax, exps, q, l);
}

// A column-major A (element (i, k) at i + k m) is a row-major n x m array
// whose columns are A's rows; a column-major B is a row-major p x n array
// whose rows are B's columns.
hipError_t pack_records(const moa_gemm_desc &d, bool two, const Fp8Workspace &w, hipStream_t st) {
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    const int64_t S = (d.n + SLAB8 - 1) / SLAB8;
    operand_records(A, d.m, d.n, S, !(d.flags & MOA_FLAG_A_COL), two, w.amaxA, w.e, w.qA, w.lA, st);
    operand_records(B, d.p, d.n, S, (d.flags & MOA_FLAG_B_COL) != 0, two, w.amaxB, w.f, w.qB, w.lB, st);
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
    return align256(4 * p) * 2 + align256(4 * m) * 2 + (two ? 2 : 1) * rec;
}

hipError_t launch_fp8(const moa_gemm_desc &d, const Plan &plan, void *ws, hipStream_t st) {
    const bool two = fp8_two_term(d);
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
    if (plan.split_k > 1) {
        float *partials = reinterpret_cast<float *>(static_cast<char *>(ws) + plan.partial_offset);
        if (two) return ring::launch_splitk<128, 128, 64, 64, 2, Fp8Mode<true>, 3>(op, plan.split_k, partials, st);
        return ring::launch_splitk<128, 128, 64, 64, 1, Fp8Mode<false>, 3>(op, plan.split_k, partials, st);
    }
    if (two) {
        switch (plan.variant) {
        case 0: return launch_shape<128, 128, 64, 64, true>(op, st);
        case 1: return launch_shape<128, 128, 64, 32, true>(op, st);
        case 2: return launch_shape<128, 128, 64, 32, true, 5>(op, st);
        case 4: return launch_shape<128, 256, 64, 64, true, 3>(op, st);
        case 5: return launch_shape<256, 128, 64, 64, true, 3>(op, st);
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

int64_t fp8_grouped_desc_bytes(int count) { return (int64_t)count * (int64_t)sizeof(Fp8Member); }

namespace {
int64_t member_bytes(const moa_gemm_desc &d, bool two) {
    const int64_t S = (d.n + SLAB8 - 1) / SLAB8;
    const int64_t rec = align256(ring::array_bytes(d.m, S)) + align256(ring::array_bytes(d.p, S));
    return align256(4 * d.m) + align256(4 * d.p) + (two ? 2 : 1) * rec;
}
int64_t header_bytes(const moa_gemm_desc *const *members, int count) {
    int64_t cols = 0;
    for (int k = 0; k < count; ++k) cols += members[k]->p;
    return align256(8 + 4 * cols);     // claim counter, then every member's column amax
}
}  // namespace

int64_t fp8_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count, bool two) {
    int64_t b = header_bytes(members, count) + align256(fp8_grouped_desc_bytes(count));
    for (int k = 0; k < count; ++k) b += member_bytes(*members[k], two);
    return b;
}

// Workspace: [counter u64 | amax of every member][member table][per member:
// e, f, record arrays]. Members are listed longest k walk first.
Fp8GroupWork fp8_grouped_layout(const moa_gemm_desc *const *members, int count, bool two, void *ws,
                                void *host_staging) {
    std::vector<int> order(count);
    for (int k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return members[a]->n > members[b]->n; });
    char *base = static_cast<char *>(ws);
    uint32_t *amax = reinterpret_cast<uint32_t *>(base + 8);
    char *cur = base + header_bytes(members, count) + align256(fp8_grouped_desc_bytes(count));
    Fp8Member *h = static_cast<Fp8Member *>(host_staging);
    Fp8GroupWork w{0, 0, 0, 2, header_bytes(members, count)};
    for (int q = 0; q < count; ++q) {
        const moa_gemm_desc &d = *members[order[q]];
        Fp8Member g;
        g.A = static_cast<const float *>(d.A);
        g.B = static_cast<const float *>(d.B);
        g.m = d.m; g.n = d.n; g.p = d.p;
        g.S = (d.n + SLAB8 - 1) / SLAB8;
        g.amaxB = amax;
        amax += d.p;
        w.clear_words += d.p;
        g.e = reinterpret_cast<int32_t *>(cur); cur += align256(4 * d.m);
        g.f = reinterpret_cast<int32_t *>(cur); cur += align256(4 * d.p);
        g.qa = reinterpret_cast<uint8_t *>(cur); cur += align256(ring::array_bytes(d.m, g.S));
        g.qb = reinterpret_cast<uint8_t *>(cur); cur += align256(ring::array_bytes(d.p, g.S));
        g.la = g.lb = nullptr;
        if (two) {
            g.la = reinterpret_cast<uint8_t *>(cur); cur += align256(ring::array_bytes(d.m, g.S));
            g.lb = reinterpret_cast<uint8_t *>(cur); cur += align256(ring::array_bytes(d.p, g.S));
        }
        g.op.a0 = g.qa; g.op.a1 = g.la;
        g.op.b0 = g.qb; g.op.b1 = g.lb;
        g.op.C = static_cast<float *>(d.C);
        g.op.row_exp = g.e;
        g.op.col_exp = g.f;
        g.op.m = d.m; g.op.p = d.p; g.op.S = g.S;
        g.op.accumulate = d.accumulate;
        g.vec_a = (d.n % 4 == 0) && ((uintptr_t)d.A % 16 == 0);
        g.vec_b = (d.p % 4 == 0) && ((uintptr_t)d.B % 16 == 0);
        g.tiles_n = (int32_t)((d.p + G_BN - 1) / G_BN);
        g.first_tile = w.tiles;
        w.tiles += ((d.m + G_BM - 1) / G_BM) * g.tiles_n;
        g.row_items = (int32_t)((d.m + 3) / 4);
        g.col_amax_x = (int32_t)((d.p + 255) / 256);
        g.scale_first = w.scale_items;
        w.scale_items += g.row_items + (int64_t)g.col_amax_x * ((d.n + COL_BAND - 1) / COL_BAND);
        g.pack_row_items = (int32_t)((padded_rows(d.m) * g.S * 4 + 255) / 256);
        g.pack_col_x = (int32_t)((d.p + 63) / 64);
        g.pack_first = w.pack_items;
        w.pack_items += g.pack_row_items + (int64_t)g.pack_col_x * (g.S > 0 ? g.S : 1);
        h[q] = g;
    }
    return w;
}

hipError_t fp8_grouped_enqueue(void *ws, int count, bool two, const Fp8GroupWork &w, hipStream_t st) {
    char *base = static_cast<char *>(ws);
    unsigned long long *counter = reinterpret_cast<unsigned long long *>(base);
    const Fp8Member *dev = reinterpret_cast<const Fp8Member *>(base + w.table_offset);
    {
        TraceScope ts(MOA_K_FP8_QUANT, st);
        hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((w.clear_words + 255) / 256)), dim3(256), 0, st,
                           reinterpret_cast<uint32_t *>(base), w.clear_words);
        if (w.scale_items > 0)
            hipLaunchKernelGGL(grouped_scales_kernel, dim3((unsigned)std::min<int64_t>(w.scale_items, 8 * kNumCUs)),
                               dim3(256), 0, st, dev, count, w.scale_items);
        if (w.pack_items > 0) {
            const dim3 grid((unsigned)std::min<int64_t>(w.pack_items, 8 * kNumCUs));
            if (two) hipLaunchKernelGGL(grouped_records_kernel<true>, grid, dim3(256), 0, st, dev, count, w.pack_items);
            else hipLaunchKernelGGL(grouped_records_kernel<false>, grid, dim3(256), 0, st, dev, count, w.pack_items);
        }
    }
    TraceScope ts(MOA_K_FP8_GROUPED, st);
    if (w.tiles > 0) {
        if (two) {
            constexpr int WM = 64, WN = 32, NST = 4;
            hipLaunchKernelGGL((fp8_grouped_kernel<true, G_BM, G_BN, WM, WN, NST>),
                               dim3((unsigned)std::min<int64_t>(w.tiles, G_PER_CU_TWO * kNumCUs)),
                               dim3(ring::Cfg<G_BM, G_BN, WM, WN, 2, NST>::THREADS), 0, st, dev, count, w.tiles,
                               counter);
        } else {
            constexpr int WM = 64, WN = 64, NST = 3;
            hipLaunchKernelGGL((fp8_grouped_kernel<false, G_BM, G_BN, WM, WN, NST>),
                               dim3((unsigned)std::min<int64_t>(w.tiles, G_PER_CU_ONE * kNumCUs)),
                               dim3(ring::Cfg<G_BM, G_BN, WM, WN, 1, NST>::THREADS), 0, st, dev, count, w.tiles,
                               counter);
        }
    }
    return hipGetLastError();
}

namespace {
// The member table straight from pinned host memory mapped into the device's
// address space (n16 16-byte words): a kernel in place of a copy-engine
// transfer and its hand-offs to and from the compute queue.
__global__ __launch_bounds__(256) void table_from_host_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                              int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}
}  // namespace

hipError_t launch_fp8_grouped(const moa_gemm_desc *const *members, int count, bool two, void *ws,
                              void *host_staging, const void *host_staging_dev, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const Fp8GroupWork w = fp8_grouped_layout(members, count, two, ws, host_staging);
    char *table = static_cast<char *>(ws) + w.table_offset;
    const int64_t bytes = fp8_grouped_desc_bytes(count);
    if (host_staging_dev) {
        const int64_t n16 = (bytes + 15) / 16;
        hipLaunchKernelGGL(table_from_host_kernel, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 64)),
                           dim3(256), 0, st, static_cast<const uint4 *>(host_staging_dev),
                           reinterpret_cast<uint4 *>(table), n16);
    } else {
        hipError_t e = hipMemcpyAsync(table, host_staging, (size_t)bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
    }
    return fp8_grouped_enqueue(ws, count, two, w, st);
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
