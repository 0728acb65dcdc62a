// FP32 matrix-core kernel: Eq. 3 with FP32 operands on v_mfma_f32_32x32x2_f32
// and FP32 accumulation. Same blocking as the split-BF16 kernel (Fig. 2: a
// BM x BN block of C per workgroup, the k extent in LDS slabs of BK whose
// block products are summed in registers).
//
// LDS row layout: one row per row of A / column of B, BK floats + 4 floats of
// pad (144 bytes for BK = 32), so consecutive rows fall in distinct 16-byte
// bank groups. Each lane half h = lane/32 owns k in [16h, 16h + 16) of a slab
// and feeds its values to 16 consecutive matrix-core steps, four per 16-byte
// LDS read (the k label inside a step is arbitrary as long as A and B agree).
#include "moa_internal.h"
#include "tile_common.h"

namespace moa {
namespace {

constexpr int BK = 32;
constexpr int ROWF = BK + 4;          // floats per LDS row (144 bytes)
constexpr int BM = 128, BN = 128, WM = 64, WN = 64;

__global__ __launch_bounds__(256) void mfma_f32_kernel(const float *__restrict__ A,
                                                       const float *__restrict__ B,
                                                       float *__restrict__ C, int64_t m,
                                                       int64_t n, int64_t p, int accumulate,
                                                       int tiles_m, int tiles_n, int vec_a) {
    constexpr int WAVES_N = BN / WN;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int CA = BM * (BK / 8) / 256;
    constexpr int CB = BN * (BK / 8) / 256;
    __shared__ __attribute__((aligned(16))) float lds[2][(BM + BN) * ROWF];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, &tm, &tn);
    const int64_t i0 = (int64_t)tm * BM;
    const int64_t j0 = (int64_t)tn * BN;

    float ra[CA][8], rb[CB][8];
    // whole blocks (the slab inside n, the block inside m and p, A vector-aligned)
    // load without per-element checks
    const bool inner = i0 + BM <= m && j0 + BN <= p && vec_a;
    auto load = [&](int64_t k0) {
        if (inner && k0 + BK <= n) {
#pragma unroll
            for (int s = 0; s < CA; ++s) {
                const int cid = t + 256 * s;
                const int row = cid % BM, kc = cid / BM;
                const float4 *src = reinterpret_cast<const float4 *>(A + (i0 + row) * n + k0 + kc * 8);
                const float4 x0 = src[0], x1 = src[1];
                ra[s][0] = x0.x; ra[s][1] = x0.y; ra[s][2] = x0.z; ra[s][3] = x0.w;
                ra[s][4] = x1.x; ra[s][5] = x1.y; ra[s][6] = x1.z; ra[s][7] = x1.w;
            }
#pragma unroll
            for (int s = 0; s < CB; ++s) {
                const int cid = t + 256 * s;
                const int col = cid % BN, kc = cid / BN;
                const float *src = B + (k0 + kc * 8) * p + j0 + col;
#pragma unroll
                for (int e = 0; e < 8; ++e) rb[s][e] = src[e * p];
            }
            return;
        }
#pragma unroll
        for (int s = 0; s < CA; ++s) {
            const int cid = t + 256 * s;
            const int row = cid % BM, kc = cid / BM;
            const int64_t i = i0 + row, k = k0 + kc * 8;
            if (i < m && vec_a && k + 8 <= n) {
                const float4 *src = reinterpret_cast<const float4 *>(A + i * n + k);
                const float4 x0 = src[0], x1 = src[1];
                ra[s][0] = x0.x; ra[s][1] = x0.y; ra[s][2] = x0.z; ra[s][3] = x0.w;
                ra[s][4] = x1.x; ra[s][5] = x1.y; ra[s][6] = x1.z; ra[s][7] = x1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    ra[s][e] = (i < m && k + e < n) ? A[i * n + k + e] : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < CB; ++s) {
            const int cid = t + 256 * s;
            const int col = cid % BN, kc = cid / BN;
            const int64_t j = j0 + col, k = k0 + kc * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                rb[s][e] = (j < p && k + e < n) ? B[(k + e) * p + j] : 0.0f;
        }
    };
    auto store = [&](int buf) {
        float *base = lds[buf];
#pragma unroll
        for (int s = 0; s < CA; ++s) {
            const int cid = t + 256 * s;
            const int row = cid % BM, kc = cid / BM;
            float4 *dst = reinterpret_cast<float4 *>(base + row * ROWF + kc * 8);
            dst[0] = make_float4(ra[s][0], ra[s][1], ra[s][2], ra[s][3]);
            dst[1] = make_float4(ra[s][4], ra[s][5], ra[s][6], ra[s][7]);
        }
#pragma unroll
        for (int s = 0; s < CB; ++s) {
            const int cid = t + 256 * s;
            const int col = cid % BN, kc = cid / BN;
            float4 *dst = reinterpret_cast<float4 *>(base + BM * ROWF + col * ROWF + kc * 8);
            dst[0] = make_float4(rb[s][0], rb[s][1], rb[s][2], rb[s][3]);
            dst[1] = make_float4(rb[s][4], rb[s][5], rb[s][6], rb[s][7]);
        }
    };

    f32x16_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int64_t nslabs = (n + BK - 1) / BK;
    if (nslabs > 0) {
        load(0);
        store(0);
        __syncthreads();
    }
    const int frag_row = lane & 31;
    const int half_k = (lane >> 5) * (BK / 2);
    for (int64_t s = 0; s < nslabs; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nslabs) load((s + 1) * BK);
        const float *la = lds[buf] + (wm * WM + frag_row) * ROWF + half_k;
        const float *lb = lds[buf] + BM * ROWF + (wn * WN + frag_row) * ROWF + half_k;
#pragma unroll
        for (int kq = 0; kq < BK / 2; kq += 4) {
            float4 av[FM], bv[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) av[a] = *reinterpret_cast<const float4 *>(la + a * 32 * ROWF + kq);
#pragma unroll
            for (int b = 0; b < FN; ++b) bv[b] = *reinterpret_cast<const float4 *>(lb + b * 32 * ROWF + kq);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            ((const float *)&av[a])[e], ((const float *)&bv[b])[e], acc[a][b], 0, 0, 0);
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
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                if (i < m) {
                    float v = acc[a][b][r];
                    if (accumulate) v += C[i * p + j];
                    C[i * p + j] = v;
                }
            }
        }
}

}  // namespace

void mfma_f32_shape(Plan *p) {
    p->variant = 0;
    p->tile_m = BM;
    p->tile_n = BN;
    p->tile_k = BK;
    p->wave_m = WM;
    p->wave_n = WN;
    p->lane_m = p->lane_n = 0;
    p->threads = 256;
    p->lds_bytes = 2 * (BM + BN) * ROWF * 4;
}

hipError_t launch_mfma_f32(const moa_gemm_desc &d, const Plan &, hipStream_t st) {
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    float *C = static_cast<float *>(d.C);
    const int tiles_m = (int)((d.m + BM - 1) / BM);
    const int tiles_n = (int)((d.p + BN - 1) / BN);
    const int vec_a = (d.n % 8 == 0) && ((uintptr_t)A % 16 == 0);
    hipLaunchKernelGGL(mfma_f32_kernel, dim3(tiles_m * tiles_n), dim3(256), 0, st, A, B, C, d.m,
                       d.n, d.p, d.accumulate, tiles_m, tiles_n, vec_a);
    return hipGetLastError();
}

}  // namespace moa
