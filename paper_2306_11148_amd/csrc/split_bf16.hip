// Split-BF16 matrix-core kernel: C = hi(A).hi(B) + hi(A).lo(B) + lo(A).hi(B)
// with FP32 accumulation, where x = hi + lo + O(2^-16 |x|) and hi, lo are
// BF16. This evaluates Eq. 3 (section "MoA Matrix Multiplication") to about
// FP32 accuracy on the BF16 matrix cores.
//
// Blocking follows the blocked form of Fig. 2: each workgroup owns a BM x BN
// block of C, walks the k extent in slabs of BK (the sigma loop broken into
// blocks), and the per-slab block products are summed in registers (the
// "addition loop" over blocks). Operands are conditioned while they are
// staged: FP32 rows of A and columns of B are read from HBM, split into
// (hi, lo) in registers and stored to LDS as k-contiguous BF16 runs, so no
// split copy of A or B is ever written to HBM.
//
// LDS row layout (one row per row of A / column of B):
//   [hi: BK bf16][lo: BK bf16][16-byte pad]  -> 144 bytes for BK = 32.
// The 9 x 16-byte pitch puts 8 consecutive rows in 8 different 16-byte bank
// groups, so the fragment reads (32 consecutive rows, one 16-byte run each)
// and the staging writes (consecutive rows) are free of bank conflicts.
#include "moa_internal.h"
#include "tile_common.h"

namespace moa {
namespace {

constexpr int BK = 32;
constexpr int ROW = 2 * BK + 8;        // bf16 elements per LDS row (144 bytes)

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void split_bf16_kernel(
    const float *__restrict__ A, const float *__restrict__ B, float *__restrict__ C,
    int64_t m, int64_t n, int64_t p, int accumulate, int tiles_m, int tiles_n, int vec_a) {
    constexpr int WAVES_N = BN / WN;
    static_assert((BM / WM) * WAVES_N == 4, "four waves");
    constexpr int FM = WM / 32, FN = WN / 32;      // 32x32 blocks per wave
    constexpr int CA = BM * (BK / 8) / 256;        // 8-element chunks per thread (A)
    constexpr int CB = BN * (BK / 8) / 256;        // (B)

    __shared__ __attribute__((aligned(16))) uint16_t lds[2][(BM + BN) * ROW];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;

    int tm, tn;
    const int total = tiles_m * tiles_n;
    tile_coords(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, 8, &tm, &tn);
    const int64_t i0 = (int64_t)tm * BM;
    const int64_t j0 = (int64_t)tn * BN;

    float ra[CA][8];
    float rb[CB][8];

    auto load = [&](int64_t k0) {
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
        uint16_t *base = lds[buf];
#pragma unroll
        for (int s = 0; s < CA; ++s) {
            const int cid = t + 256 * s;
            const int row = cid % BM, kc = cid / BM;
            uint4 hi, lo;
            split_pair(ra[s][0], ra[s][1], &hi.x, &lo.x);
            split_pair(ra[s][2], ra[s][3], &hi.y, &lo.y);
            split_pair(ra[s][4], ra[s][5], &hi.z, &lo.z);
            split_pair(ra[s][6], ra[s][7], &hi.w, &lo.w);
            *reinterpret_cast<uint4 *>(base + row * ROW + kc * 8) = hi;
            *reinterpret_cast<uint4 *>(base + row * ROW + BK + kc * 8) = lo;
        }
#pragma unroll
        for (int s = 0; s < CB; ++s) {
            const int cid = t + 256 * s;
            const int col = cid % BN, kc = cid / BN;
            uint4 hi, lo;
            split_pair(rb[s][0], rb[s][1], &hi.x, &lo.x);
            split_pair(rb[s][2], rb[s][3], &hi.y, &lo.y);
            split_pair(rb[s][4], rb[s][5], &hi.z, &lo.z);
            split_pair(rb[s][6], rb[s][7], &hi.w, &lo.w);
            uint16_t *bb = base + BM * ROW;
            *reinterpret_cast<uint4 *>(bb + col * ROW + kc * 8) = hi;
            *reinterpret_cast<uint4 *>(bb + col * ROW + BK + kc * 8) = lo;
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
    const int frag_k = (lane >> 5) * 8;
    for (int64_t s = 0; s < nslabs; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nslabs) load((s + 1) * BK);
        const uint16_t *la = lds[buf] + (wm * WM + frag_row) * ROW + frag_k;
        const uint16_t *lb = lds[buf] + BM * ROW + (wn * WN + frag_row) * ROW + frag_k;
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8_t ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                ah[a] = *reinterpret_cast<const bf16x8_t *>(la + a * 32 * ROW + ks);
                al[a] = *reinterpret_cast<const bf16x8_t *>(la + a * 32 * ROW + BK + ks);
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                bh[b] = *reinterpret_cast<const bf16x8_t *>(lb + b * 32 * ROW + ks);
                bl[b] = *reinterpret_cast<const bf16x8_t *>(lb + b * 32 * ROW + BK + ks);
            }
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        if (s + 1 < nslabs) store(buf ^ 1);
        __syncthreads();
    }

    // Epilogue: register r of lane l holds C[8(r/4) + 4(l/32) + r%4][l%32] of
    // each 32x32 block; 32 lanes write one 128-byte run of a row of C.
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

// Standalone conditioning kernel: hi/lo planes of a row-major FP32 array.
__global__ __launch_bounds__(256) void split_only_kernel(const float *__restrict__ X, int64_t count,
                                                         uint16_t *__restrict__ hi,
                                                         uint16_t *__restrict__ lo) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 2;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; t < count; t += stride) {
        const float x0 = X[t];
        const float x1 = (t + 1 < count) ? X[t + 1] : 0.0f;
        uint32_t h, l;
        split_pair(x0, x1, &h, &l);
        hi[t] = (uint16_t)(h & 0xFFFF);
        lo[t] = (uint16_t)(l & 0xFFFF);
        if (t + 1 < count) {
            hi[t + 1] = (uint16_t)(h >> 16);
            lo[t + 1] = (uint16_t)(l >> 16);
        }
    }
}

struct SplitShape { int bm, bn, wm, wn; };
constexpr SplitShape kSplit[] = {{128, 128, 64, 64}, {256, 256, 128, 128}};

template <int BM, int BN, int WM, int WN>
hipError_t launch_shape(const moa_gemm_desc &d, hipStream_t st) {
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    float *C = static_cast<float *>(d.C);
    const int tiles_m = (int)((d.m + BM - 1) / BM);
    const int tiles_n = (int)((d.p + BN - 1) / BN);
    const int vec_a = (d.n % 8 == 0) && ((uintptr_t)A % 16 == 0);
    hipLaunchKernelGGL((split_bf16_kernel<BM, BN, WM, WN>), dim3(tiles_m * tiles_n), dim3(256), 0,
                       st, A, B, C, d.m, d.n, d.p, d.accumulate, tiles_m, tiles_n, vec_a);
    return hipGetLastError();
}

}  // namespace

int split_bf16_variant_count() { return (int)(sizeof(kSplit) / sizeof(kSplit[0])); }

void split_bf16_shape(int v, Plan *p) {
    const SplitShape s = kSplit[v];
    p->variant = v;
    p->tile_m = s.bm;
    p->tile_n = s.bn;
    p->tile_k = BK;
    p->wave_m = s.wm;
    p->wave_n = s.wn;
    p->lane_m = p->lane_n = 0;
    p->threads = 256;
    p->lds_bytes = 2 * (s.bm + s.bn) * ROW * 2;
}

hipError_t launch_split_bf16(const moa_gemm_desc &d, const Plan &plan, hipStream_t st) {
    switch (plan.variant) {
    case 0: return launch_shape<128, 128, 64, 64>(d, st);
    default: return launch_shape<256, 256, 128, 128>(d, st);
    }
}

hipError_t launch_split_only(const float *X, int64_t count, uint16_t *hi, uint16_t *lo,
                             hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(split_only_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, count, hi, lo);
    return hipGetLastError();
}

}  // namespace moa
