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
//
// Conditioning kernels (HBM-bound): row amax of A and column amax of B
// (atomic max on the bit patterns of |x|, which order like unsigned ints),
// then quantisation of A in place order and of B into a k-contiguous
// (transposed) copy, both in a stream-ordered workspace. The GEMM kernel uses
// the blocking of Fig. 2 with v_mfma_f32_32x32x64_f8f6f4 steps.
#include "moa_internal.h"
#include "tile_common.h"

namespace moa {
namespace {

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

// One wave per row of A: amax of |A[i, :]| -> amax bits.
__global__ __launch_bounds__(256) void row_amax_kernel(const float *__restrict__ A, int64_t m,
                                                       int64_t n, uint32_t *__restrict__ amax) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    const float *row = A + i * n;
    float mx = 0.0f;
    for (int64_t k = lane; k < n; k += 64) mx = fmaxf(mx, fabsf(row[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) amax[i] = __float_as_uint(mx);
}

// Column amax of B: each thread takes one column over a 64-row band.
__global__ __launch_bounds__(256) void col_amax_kernel(const float *__restrict__ B, int64_t n,
                                                       int64_t p, uint32_t *__restrict__ amax) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.y * 64;
    if (j >= p) return;
    float mx = 0.0f;
    const int64_t k1 = min(n, k0 + 64);
    for (int64_t k = k0; k < k1; ++k) mx = fmaxf(mx, fabsf(B[k * p + j]));
    atomicMax(&amax[j], __float_as_uint(mx));
}

// qA (row-major, like A): 4 consecutive elements per thread.
__global__ __launch_bounds__(256) void quant_rows_kernel(const float *__restrict__ A, int64_t m,
                                                         int64_t n, const uint32_t *__restrict__ amax,
                                                         int two_term, int32_t *__restrict__ e_out,
                                                         uint8_t *__restrict__ q,
                                                         uint8_t *__restrict__ l) {
    const int64_t i = blockIdx.x;
    const int64_t k = ((int64_t)blockIdx.y * 256 + threadIdx.x) * 4;
    const int e = pow2_exponent(__uint_as_float(amax[i]));
    if (blockIdx.y == 0 && threadIdx.x == 0 && e_out) e_out[i] = e;
    if (k >= n) return;
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (k + t < n) ? ldexpf(A[i * n + k + t], e) : 0.0f;
    uint32_t hi, lo = 0;
    quant4(v, two_term != 0, &hi, &lo);
    uint8_t *qd = q + i * n + k;
    uint8_t *ld = l ? l + i * n + k : nullptr;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (k + t < n) {
            qd[t] = (uint8_t)(hi >> (8 * t));
            if (two_term) ld[t] = (uint8_t)(lo >> (8 * t));
        }
}

// qB for B (n x p). transposed == 0: row-major n x p like B (the exposed
// conditioning call). transposed != 0: p x n, k-contiguous per column (the
// GEMM operand). A 64 x 64 block per workgroup goes through LDS so that both
// the reads of B rows and the writes of the transposed rows are contiguous.
__global__ __launch_bounds__(256) void quant_cols_kernel(const float *__restrict__ B, int64_t n,
                                                         int64_t p, const uint32_t *__restrict__ amax,
                                                         int two_term, int transposed,
                                                         int32_t *__restrict__ f_out,
                                                         uint8_t *__restrict__ q,
                                                         uint8_t *__restrict__ l) {
    __shared__ uint8_t tq[64][64 + 4];
    __shared__ uint8_t tl[64][64 + 4];
    const int64_t k0 = (int64_t)blockIdx.y * 64, jb = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 15;      // 4 columns each
    const int ty = threadIdx.x >> 4;      // 16 rows, 4 passes
    const int64_t j = jb + tx * 4;
    int f[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f[t] = (j + t < p) ? pow2_exponent(__uint_as_float(amax[j + t])) : 0;
        if (f_out && blockIdx.y == 0 && ty == 0 && j + t < p) f_out[j + t] = f[t];
    }
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int kk = ty + 16 * pass;
        const int64_t k = k0 + kk;
        float v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            v[t] = (k < n && j + t < p) ? ldexpf(B[k * p + j + t], f[t]) : 0.0f;
        uint32_t hi, lo = 0;
        quant4(v, two_term != 0, &hi, &lo);
        if (!transposed) {
            if (k < n) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (j + t < p) {
                        q[k * p + j + t] = (uint8_t)(hi >> (8 * t));
                        if (two_term) l[k * p + j + t] = (uint8_t)(lo >> (8 * t));
                    }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                tq[tx * 4 + t][kk] = (uint8_t)(hi >> (8 * t));
                tl[tx * 4 + t][kk] = (uint8_t)(lo >> (8 * t));
            }
        }
    }
    if (!transposed) return;
    __syncthreads();
    // write 64 columns x 64 k: thread -> (column jj, 16-byte run of k)
    const int jj = threadIdx.x >> 2, run = (threadIdx.x & 3) * 16;
    const int64_t jo = jb + jj;
    if (jo >= p) return;
    for (int b = 0; b < 16; ++b) {
        const int64_t k = k0 + run + b;
        if (k < n) {
            q[jo * n + k] = tq[jj][run + b];
            if (two_term) l[jo * n + k] = tl[jj][run + b];
        }
    }
}

// ---------------------------------------------------------------- GEMM ----
// 32 consecutive E4M3 codes of one fragment row from LDS (16-byte aligned).
__device__ __forceinline__ i32x8_t frag32(const uint8_t *p) {
    const uint4 lo = *reinterpret_cast<const uint4 *>(p);
    const uint4 hi = *reinterpret_cast<const uint4 *>(p + 16);
    i32x8_t v;
    v[0] = (int)lo.x; v[1] = (int)lo.y; v[2] = (int)lo.z; v[3] = (int)lo.w;
    v[4] = (int)hi.x; v[5] = (int)hi.y; v[6] = (int)hi.z; v[7] = (int)hi.w;
    return v;
}

constexpr int BK8 = 128;                 // k per slab (bytes of E4M3)
// E8M0 block scale 2^(127-127) = 1 for both operands of the scaled
// matrix-core step (0 would mean 2^-127).
constexpr int kScaleOne = 0x7f;
constexpr int BM = 128, BN = 128, WM = 64, WN = 64;

template <bool TWO>
__global__ __launch_bounds__(256) void fp8_gemm_kernel(
    const uint8_t *__restrict__ qA, const uint8_t *__restrict__ lA, const int32_t *__restrict__ e,
    const uint8_t *__restrict__ qBt, const uint8_t *__restrict__ lBt, const int32_t *__restrict__ f,
    float *__restrict__ C, int64_t m, int64_t n, int64_t p, int accumulate, int tiles_m,
    int tiles_n, int vec) {
    // LDS row: [hi: 128 codes][lo: 128 codes, two-term only][16-byte pad]
    constexpr int ROWB = (TWO ? 2 * BK8 : BK8) + 16;
    constexpr int FM = WM / 32, FN = WN / 32, WAVES_N = BN / WN;
    constexpr int CHUNKS = (BM + BN) * (BK8 / 16);   // 16-byte chunks per plane
    constexpr int CPT = CHUNKS / 256;
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][(BM + BN) * ROWB];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, &tm, &tn);
    const int64_t i0 = (int64_t)tm * BM, j0 = (int64_t)tn * BN;

    uint4 rh[CPT], rl[TWO ? CPT : 1];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int s = 0; s < CPT; ++s) {
            const int cid = t + 256 * s;
            const int row = cid % (BM + BN), kc = cid / (BM + BN);
            const bool is_a = row < BM;
            const int64_t r = is_a ? i0 + row : j0 + (row - BM);
            const int64_t lim = is_a ? m : p;
            const uint8_t *src = is_a ? qA : qBt;
            const uint8_t *srcl = is_a ? lA : lBt;
            const int64_t k = k0 + kc * 16;
            uint4 h = make_uint4(0, 0, 0, 0), lo = make_uint4(0, 0, 0, 0);
            if (r < lim) {
                if (vec && k + 16 <= n) {
                    h = *reinterpret_cast<const uint4 *>(src + r * n + k);
                    if (TWO) lo = *reinterpret_cast<const uint4 *>(srcl + r * n + k);
                } else {
                    uint8_t *hb = reinterpret_cast<uint8_t *>(&h);
                    uint8_t *lb = reinterpret_cast<uint8_t *>(&lo);
                    for (int b = 0; b < 16; ++b)
                        if (k + b < n) {
                            hb[b] = src[r * n + k + b];
                            if (TWO) lb[b] = srcl[r * n + k + b];
                        }
                }
            }
            rh[s] = h;
            if (TWO) rl[s] = lo;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int s = 0; s < CPT; ++s) {
            const int cid = t + 256 * s;
            const int row = cid % (BM + BN), kc = cid / (BM + BN);
            *reinterpret_cast<uint4 *>(&lds[buf][row * ROWB + kc * 16]) = rh[s];
            if (TWO) *reinterpret_cast<uint4 *>(&lds[buf][row * ROWB + BK8 + kc * 16]) = rl[s];
        }
    };

    f32x16_t acc[FM][FN], acx[TWO ? FM : 1][TWO ? FN : 1];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    if (TWO) {
#pragma unroll
        for (int a = 0; a < (TWO ? FM : 1); ++a)
#pragma unroll
            for (int b = 0; b < (TWO ? FN : 1); ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acx[a][b][r] = 0.0f;
    }

    const int64_t nslabs = (n + BK8 - 1) / BK8;
    if (nslabs > 0) {
        load(0);
        store(0);
        __syncthreads();
    }
    const int frag_row = lane & 31, frag_k = (lane >> 5) * 32;
    for (int64_t s = 0; s < nslabs; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nslabs) load((s + 1) * BK8);
        const uint8_t *la = &lds[buf][(wm * WM + frag_row) * ROWB + frag_k];
        const uint8_t *lb = &lds[buf][(BM + wn * WN + frag_row) * ROWB + frag_k];
#pragma unroll
        for (int ks = 0; ks < BK8; ks += 64) {
            i32x8_t ah[FM], bh[FN], al[TWO ? FM : 1], bl[TWO ? FN : 1];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                ah[a] = frag32(la + a * 32 * ROWB + ks);
                if (TWO) al[a] = frag32(la + a * 32 * ROWB + BK8 + ks);
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                bh[b] = frag32(lb + b * 32 * ROWB + ks);
                if (TWO) bl[b] = frag32(lb + b * 32 * ROWB + BK8 + ks);
            }
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        ah[a], bh[b], acc[a][b], 0, 0, 0, kScaleOne, 0, kScaleOne);
                    if (TWO) {
                        acx[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            ah[a], bl[b], acx[a][b], 0, 0, 0, kScaleOne, 0, kScaleOne);
                        acx[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            al[a], bh[b], acx[a][b], 0, 0, 0, kScaleOne, 0, kScaleOne);
                    }
                }
        }
        if (s + 1 < nslabs) store(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t j = j0 + wn * WN + b * 32 + (lane & 31);
            if (j >= p) continue;
            const int fj = f[j];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                if (i < m) {
                    float v = acc[a][b][r];
                    if (TWO) v += ldexpf(acx[a][b][r], -4);
                    v = ldexpf(v, -(e[i] + fj));
                    if (accumulate) v += C[i * p + j];
                    C[i * p + j] = v;
                }
            }
        }
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Fp8Workspace {
    uint32_t *amaxA, *amaxB;
    int32_t *e, *f;
    uint8_t *qA, *lA, *qBt, *lBt;
};

Fp8Workspace carve(void *ws, int64_t m, int64_t n, int64_t p, bool two) {
    char *c = static_cast<char *>(ws);
    Fp8Workspace w;
    w.amaxA = reinterpret_cast<uint32_t *>(c); c += align256(4 * m);
    w.amaxB = reinterpret_cast<uint32_t *>(c); c += align256(4 * p);
    w.e = reinterpret_cast<int32_t *>(c); c += align256(4 * m);
    w.f = reinterpret_cast<int32_t *>(c); c += align256(4 * p);
    w.qA = reinterpret_cast<uint8_t *>(c); c += align256(m * n);
    w.qBt = reinterpret_cast<uint8_t *>(c); c += align256(n * p);
    w.lA = two ? reinterpret_cast<uint8_t *>(c) : nullptr; c += two ? align256(m * n) : 0;
    w.lBt = two ? reinterpret_cast<uint8_t *>(c) : nullptr;
    return w;
}

hipError_t conditioning(const float *A, int64_t m, int64_t n, const float *B, int64_t p, bool two,
                        uint32_t *amaxA, uint32_t *amaxB, int32_t *e, uint8_t *qA, uint8_t *lA,
                        int32_t *f, uint8_t *qB, uint8_t *lB, bool transposed, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, amaxA, m);
    if (p > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, amaxB, p);
    if (m > 0 && n > 0)
        hipLaunchKernelGGL(row_amax_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, A, m, n, amaxA);
    if (p > 0 && n > 0)
        hipLaunchKernelGGL(col_amax_kernel, dim3((unsigned)((p + 255) / 256), (unsigned)((n + 63) / 64)),
                           dim3(256), 0, st, B, n, p, amaxB);
    if (m > 0)
        hipLaunchKernelGGL(quant_rows_kernel, dim3((unsigned)m, (unsigned)((n + 1023) / 1024 > 0 ? (n + 1023) / 1024 : 1)),
                           dim3(256), 0, st, A, m, n, amaxA, (int)two, e, qA, lA);
    if (p > 0)
        hipLaunchKernelGGL(quant_cols_kernel, dim3((unsigned)((p + 63) / 64), (unsigned)((n + 63) / 64 > 0 ? (n + 63) / 64 : 1)),
                           dim3(256), 0, st, B, n, p, amaxB, (int)two, (int)transposed, f, qB, lB);
    return hipGetLastError();
}

}  // namespace

void fp8_shape(bool two, Plan *p) {
    p->variant = two ? 1 : 0;
    p->tile_m = BM;
    p->tile_n = BN;
    p->tile_k = BK8;
    p->wave_m = WM;
    p->wave_n = WN;
    p->lane_m = p->lane_n = 0;
    p->threads = 256;
    p->lds_bytes = 2 * (BM + BN) * ((two ? 2 * BK8 : BK8) + 16);
}

int64_t fp8_workspace_bytes(int64_t m, int64_t n, int64_t p, bool two) {
    int64_t b = align256(4 * m) * 2 + align256(4 * p) * 2 + align256(m * n) + align256(n * p);
    if (two) b += align256(m * n) + align256(n * p);
    return b;
}

hipError_t launch_fp8(const moa_gemm_desc &d, const Plan &plan, void *ws, hipStream_t st) {
    const bool two = (d.flags & MOA_FLAG_FP8_TWO_TERM) != 0;
    const Fp8Workspace w = carve(ws, d.m, d.n, d.p, two);
    hipError_t err;
    {
        TraceScope ts(MOA_K_FP8_QUANT, st);
        err = conditioning(static_cast<const float *>(d.A), d.m, d.n, static_cast<const float *>(d.B),
                           d.p, two, w.amaxA, w.amaxB, w.e, w.qA, w.lA, w.f, w.qBt, w.lBt, true, st);
    }
    if (err != hipSuccess) return err;
    TraceScope ts(two ? MOA_K_FP8_2TERM : MOA_K_FP8, st);
    const int tiles_m = (int)((d.m + BM - 1) / BM), tiles_n = (int)((d.p + BN - 1) / BN);
    const int vec = (d.n % 16 == 0);
    float *C = static_cast<float *>(d.C);
    if (two)
        hipLaunchKernelGGL(fp8_gemm_kernel<true>, dim3(tiles_m * tiles_n), dim3(256), 0, st, w.qA, w.lA,
                           w.e, w.qBt, w.lBt, w.f, C, d.m, d.n, d.p, d.accumulate, tiles_m, tiles_n, vec);
    else
        hipLaunchKernelGGL(fp8_gemm_kernel<false>, dim3(tiles_m * tiles_n), dim3(256), 0, st, w.qA, w.lA,
                           w.e, w.qBt, w.lBt, w.f, C, d.m, d.n, d.p, d.accumulate, tiles_m, tiles_n, vec);
    (void)plan;
    return hipGetLastError();
}

hipError_t launch_quantise_fp8(const float *A, int64_t m, int64_t n, const float *B, int64_t p,
                               bool two, int32_t *e, uint8_t *qA, uint8_t *lA, int32_t *f,
                               uint8_t *qB, uint8_t *lB, uint32_t *amax, hipStream_t st) {
    return conditioning(A, m, n, B, p, two, amax, amax + m, e, qA, lA, f, qB, lB, false, st);
}

}  // namespace moa
