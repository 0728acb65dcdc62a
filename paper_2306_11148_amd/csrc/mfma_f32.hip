// FP32 matrix-core kernels: Eq. 3 with FP32 operands on v_mfma_f32_32x32x2_f32
// and FP32 accumulation, with the blocking of Fig. 2 (a BM x BN block of C per
// workgroup, the k extent in slabs whose block products are summed in
// registers). Two forms:
//  * record ring (the default): A's rows and B's columns are first copied into
//    64-byte records of 16 FP32 values (the record-tile layout of the
//    split-BF16 path, B transposed) and the contraction runs the shared
//    direct-to-LDS ring (ring_gemm.h) with an FP32 fragment mode;
//  * register-staged (no workspace; used where a call may not take scratch,
//    such as prepared groups): the kernel below.
//
// LDS row layout: one row per row of A / column of B, BK floats + 4 floats of
// pad (144 bytes for BK = 32), so consecutive rows fall in distinct 16-byte
// bank groups. Each lane half h = lane/32 owns k in [16h, 16h + 16) of a slab
// and feeds its values to 16 consecutive matrix-core steps, four per 16-byte
// LDS read (the k label inside a step is arbitrary as long as A and B agree).
#include <algorithm>

#include "moa_internal.h"
#include "ring_gemm.h"
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

    // the accumulate form reads a block's 16 values of C before any store
    auto epilogue = [&](auto acc_form) {
        constexpr bool ACC = decltype(acc_form)::value;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int64_t j = j0 + wn * WN + b * 32 + (lane & 31);
                if (j >= p) continue;
                float old[16];
                if constexpr (ACC) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                        if (i < m) old[r] = C[i * p + j];
                    }
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                    if (i < m) {
                        float v = acc[a][b][r];
                        if constexpr (ACC) v += old[r];
                        C[i * p + j] = v;
                    }
                }
            }
    };
    if (accumulate)
        epilogue(std::true_type{});
    else
        epilogue(std::false_type{});
}

// ------------------------------------------------------------ record ring --
using ring::GROUP;
using ring::padded_rows;
constexpr int SLAB32 = 16;                 // k per FP32 record: 16 floats = 64 bytes
static_assert(SLAB32 * 4 == ring::REC_BYTES, "one record holds one slab of one row");

// Rows of X (rows x K, row-major) -> records; chunk q = 8 values, half a record.
// Consecutive chunks fill one KiB record tile contiguously.
__global__ __launch_bounds__(256) void f32_rows_kernel(const float *__restrict__ X, int64_t rows, int64_t K,
                                                       int64_t S, int vec, uint8_t *__restrict__ P) {
    const int64_t chunks = padded_rows(rows) * S * 2;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256) {
        const int c = (int)(q & 1);
        const int64_t rr = (q >> 1) % GROUP, gs = (q >> 1) / GROUP;
        const int64_t s = gs % S, r = (gs / S) * GROUP + rr;
        const int64_t k = s * SLAB32 + c * 8;
        float4 x0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), x1 = x0;
        if (r < rows) {
            if (vec && k + 8 <= K) {
                const float4 *src = reinterpret_cast<const float4 *>(X + r * K + k);
                x0 = src[0];
                x1 = src[1];
            } else {
                float *e0 = reinterpret_cast<float *>(&x0), *e1 = reinterpret_cast<float *>(&x1);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (k + e < K) e0[e] = X[r * K + k + e];
                    if (k + 4 + e < K) e1[e] = X[r * K + k + 4 + e];
                }
            }
        }
        float4 *dst = reinterpret_cast<float4 *>(P + ring::rec_byte(r, s, S) + c * 32);
        dst[0] = x0;
        dst[1] = x1;
    }
}

// Columns of X (K x cols, row-major) -> records (transposed): 64 columns x 64 k
// (four slabs) per step through LDS; each thread then writes two half records,
// so that a wave's 16-byte stores fill half of every record of two row tiles.
// Columns past `cols` get zero records. All 256 threads take part.
__global__ __launch_bounds__(256) void f32_cols_kernel(const float *__restrict__ X, int64_t K, int64_t cols,
                                                       int64_t S, int vec, uint8_t *__restrict__ P) {
    __shared__ __attribute__((aligned(16))) float tile[4 * SLAB32][64 + 4];
    const int t = threadIdx.x;
    const int64_t bx = blockIdx.x;
    const int64_t by_count = (S + 3) / 4;
    for (int64_t by = blockIdx.y; by < by_count; by += gridDim.y) {
        const int64_t j = bx * 64 + (t & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = (t >> 4) + 16 * i;
            const int64_t k = by * 4 * SLAB32 + kk;
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (k < K) {
                if (vec && j + 4 <= cols) {
                    v = *reinterpret_cast<const float4 *>(X + k * cols + j);
                } else {
                    float *e = reinterpret_cast<float *>(&v);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (j + q < cols) e[q] = X[k * cols + j + q];
                }
            }
            *reinterpret_cast<float4 *>(&tile[kk][(t & 15) * 4]) = v;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = t + 256 * h;
            const int c = u & 1, jj = (u >> 1) & 63, part = u >> 7;
            const int64_t col = bx * 64 + jj, s = by * 4 + part;
            if (col < padded_rows(cols) && s < S) {
                const int kb = part * SLAB32 + c * 8;
                float4 *dst = reinterpret_cast<float4 *>(P + ring::rec_byte(col, s, S) + c * 32);
                dst[0] = make_float4(tile[kb][jj], tile[kb + 1][jj], tile[kb + 2][jj], tile[kb + 3][jj]);
                dst[1] = make_float4(tile[kb + 4][jj], tile[kb + 5][jj], tile[kb + 6][jj], tile[kb + 7][jj]);
            }
        }
        __syncthreads();                         // tile free for the next block
    }
}

// Fragments of one slab: lane half h = l/32 holds k in [8h, 8h + 8) of its
// row (record chunks 2h, 2h + 1); matrix-core step j pairs k = j (lanes 0-31)
// with k = 8 + j (lanes 32-63), so the eight steps cover the slab's 16 k.
struct F32Mode {
    static constexpr bool SCALED = false;
    template <int FM, int FN> struct Frags { float4 a[FM][2], b[FN][2]; };

    template <int BM, int BN, int FM, int FN>
    static __device__ __forceinline__ void read(const uint8_t *buf, int a_row, int b_row, int half,
                                                Frags<FM, FN> &f) {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            f.a[a][0] = ring::lds_chunk<float4>(buf, a_row + a * 32, 2 * half);
            f.a[a][1] = ring::lds_chunk<float4>(buf, a_row + a * 32, 2 * half + 1);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            f.b[b][0] = ring::lds_chunk<float4>(buf, b_row + b * 32, 2 * half);
            f.b[b][1] = ring::lds_chunk<float4>(buf, b_row + b * 32, 2 * half + 1);
        }
    }

    template <int FM, int FN>
    static __device__ __forceinline__ void mma(const Frags<FM, FN> &f, f32x16_t (&acc)[FM][FN]) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(((const float *)&f.a[a][j / 4])[j % 4],
                                                                     ((const float *)&f.b[b][j / 4])[j % 4],
                                                                     acc[a][b], 0, 0, 0);
    }
};

template <int RBM, int RBN, int RWM, int RWN>
hipError_t launch_ring(const moa_gemm_desc &d, const uint8_t *Ap, const uint8_t *Bp, int64_t S, hipStream_t st) {
    ring::Operands op;
    op.a0 = Ap; op.a1 = nullptr;
    op.b0 = Bp; op.b1 = nullptr;
    op.C = static_cast<float *>(d.C);
    op.row_exp = op.col_exp = nullptr;
    op.m = d.m; op.p = d.p; op.S = S;
    op.accumulate = d.accumulate;
    const int tiles_m = (int)((d.m + RBM - 1) / RBM);
    const int tiles_n = (int)((d.p + RBN - 1) / RBN);
    hipLaunchKernelGGL((ring::single_kernel<RBM, RBN, RWM, RWN, 1, F32Mode, 3>), dim3(tiles_m * tiles_n),
                       dim3(ring::Cfg<RBM, RBN, RWM, RWN, 1, 3>::THREADS), 0, st, op, tiles_m, tiles_n);
    return hipGetLastError();
}

struct F32Shape { int bm, bn, wm, wn; bool ring; };
// 3 and 4: rectangular blocks of four 128 x 64 / 64 x 128 waves, two per CU
constexpr F32Shape kF32Mfma[] = {{128, 128, 64, 64, true}, {256, 256, 128, 64, true}, {BM, BN, WM, WN, false},
                                 {256, 128, 128, 64, true}, {128, 256, 64, 128, true}};
constexpr int kRegisterStaged = 2;         // the variant without workspace

}  // namespace

int mfma_f32_variant_count() { return (int)(sizeof(kF32Mfma) / sizeof(kF32Mfma[0])); }
int mfma_f32_staged_variant() { return kRegisterStaged; }

// 256 x 256 blocks once they give every CU a block, else 128 x 128; the
// rectangular blocks when 256 x 256 ones fill more than one round of the CUs
// but leave the last round less than 40% full (as on the split-BF16 path).
int mfma_f32_default_variant(int64_t m, int64_t p) {
    const int64_t big = ((m + 255) / 256) * ((p + 255) / 256);
    if (big < kNumCUs) return 0;
    const int64_t tail = big % kNumCUs;
    if (big > kNumCUs && tail != 0 && 10 * tail < 4 * kNumCUs) return p >= m ? 4 : 3;
    return 1;
}

int64_t mfma_f32_workspace_bytes(int64_t m, int64_t n, int64_t p, int v) {
    if (!kF32Mfma[v].ring) return 0;
    const int64_t S = (n + SLAB32 - 1) / SLAB32;
    return ring::array_bytes(m, S) + ring::array_bytes(p, S);
}

void mfma_f32_shape(int v, Plan *p) {
    const F32Shape s = kF32Mfma[v];
    p->variant = v;
    p->tile_m = s.bm;
    p->tile_n = s.bn;
    p->tile_k = s.ring ? SLAB32 : BK;
    p->wave_m = s.wm;
    p->wave_n = s.wn;
    p->lane_m = p->lane_n = 0;
    p->threads = (s.bm / s.wm) * (s.bn / s.wn) * 64;
    p->lds_bytes = s.ring ? 3 * (s.bm + s.bn) * ring::REC_BYTES : 2 * (BM + BN) * ROWF * 4;
}

hipError_t launch_mfma_f32(const moa_gemm_desc &d, const Plan &plan, void *ws, hipStream_t st) {
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    float *C = static_cast<float *>(d.C);
    if (kF32Mfma[plan.variant].ring) {
        const int64_t S = (d.n + SLAB32 - 1) / SLAB32;
        uint8_t *Ap = static_cast<uint8_t *>(ws);
        uint8_t *Bp = Ap + ring::array_bytes(d.m, S);
        if (S > 0) {
            // A's rows and B's columns as records. A column-major A (element
            // (i, k) at i + k m) is a row-major n x m array whose columns are
            // A's rows; a column-major B is a row-major p x n array whose rows
            // are B's columns.
            auto rows = [&](const float *X, int64_t r, uint8_t *P) {
                const int vec = (d.n % 8 == 0) && ((uintptr_t)X % 16 == 0);
                const int64_t rb = std::min<int64_t>((padded_rows(r) * S * 2 + 255) / 256, 65536);
                hipLaunchKernelGGL(f32_rows_kernel, dim3((unsigned)rb), dim3(256), 0, st, X, r, d.n, S, vec, P);
            };
            auto cols = [&](const float *X, int64_t c, uint8_t *P) {
                const int vec = (c % 4 == 0) && ((uintptr_t)X % 16 == 0);
                const int64_t by = std::min<int64_t>((S + 3) / 4, 65535);
                hipLaunchKernelGGL(f32_cols_kernel, dim3((unsigned)((c + 63) / 64), (unsigned)by), dim3(256), 0, st,
                                   X, d.n, c, S, vec, P);
            };
            if (d.flags & MOA_FLAG_A_COL) cols(A, d.m, Ap); else rows(A, d.m, Ap);
            if (d.flags & MOA_FLAG_B_COL) rows(B, d.p, Bp); else cols(B, d.p, Bp);
        }
        switch (plan.variant) {
        case 1: return launch_ring<256, 256, 128, 64>(d, Ap, Bp, S, st);
        case 3: return launch_ring<256, 128, 128, 64>(d, Ap, Bp, S, st);
        case 4: return launch_ring<128, 256, 64, 128>(d, Ap, Bp, S, st);
        default: return launch_ring<128, 128, 64, 64>(d, Ap, Bp, S, st);
        }
    }
    const int tiles_m = (int)((d.m + BM - 1) / BM);
    const int tiles_n = (int)((d.p + BN - 1) / BN);
    const int vec_a = (d.n % 8 == 0) && ((uintptr_t)A % 16 == 0);
    hipLaunchKernelGGL(mfma_f32_kernel, dim3(tiles_m * tiles_n), dim3(256), 0, st, A, B, C, d.m,
                       d.n, d.p, d.accumulate, tiles_m, tiles_n, vec_a);
    return hipGetLastError();
}

}  // namespace moa
