// Split-BF16 matrix-core path: C = hi(A).hi(B) + hi(A).lo(B) + lo(A).hi(B)
// with FP32 accumulation, where x = hi + lo + O(2^-16 |x|), hi = RNE_bf16(x),
// lo = RNE_bf16(x - hi). This evaluates Eq. 3 (section "MoA Matrix
// Multiplication") to about FP32 accuracy on the BF16 matrix cores.
//
// Two stages.
//
// 1. Conditioning (HBM-bound): A and B are rewritten as record tiles (layout
//    in ring_gemm.h). The k extent is cut into slabs of 16 (the sigma loop
//    broken into blocks, section "Dimension Lifting to Machine Coordinates");
//    for every row i of A and every column j of B, slab s becomes one
//    contiguous 64-byte record
//        [hi of x[16s .. 16s+15] (16 bf16)][lo of the same (16 bf16)]
//    zero-padded past n. B is transposed on the way (column j of B becomes
//    record row j), so both operands are k-contiguous.
//
// 2. Contraction (matrix-core bound): the record-tile ring of ring_gemm.h
//    (blocked form of Fig. 2) with three BF16 matrix-core steps per slab and
//    block pair, FP32 accumulation.
#include <algorithm>
#include <cstring>
#include <vector>

#include "moa_internal.h"
#include "ring_gemm.h"
#include "tile_common.h"

namespace moa {
namespace {

using ring::GROUP;
using ring::padded_rows;
using ring::REC_BYTES;

constexpr int SLAB = 16;                  // k per record: [hi 16 bf16][lo 16 bf16] = 64 bytes
static_assert(REC_BYTES == 2 * SLAB * 2, "one record holds hi and lo of one slab");

// ---------------------------------------------------------------- stage 1 --

// Rows of X (rows x K, row-major) -> records: chunk q = 8 k values of one
// record (2 chunks per record).
__device__ __forceinline__ void pack_rows_chunk(const float *__restrict__ X, int64_t rows, int64_t K,
                                                int64_t S, int vec, uint8_t *__restrict__ P,
                                                int64_t q) {
    // q -> (row tile g, slab s, row rr in the tile, chunk c): consecutive
    // threads fill one KiB tile contiguously
    const int c = (int)(q & 1);
    const int64_t rr = (q >> 1) % GROUP;
    const int64_t gs = (q >> 1) / GROUP;
    const int64_t s = gs % S, g = gs / S;
    const int64_t r = g * GROUP + rr;
    const int64_t k = s * SLAB + c * 8;
    float x[8];
    if (r >= rows) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.0f;
    } else if (vec && k + 8 <= K) {
        const float4 *src = reinterpret_cast<const float4 *>(X + r * K + k);
        const float4 a = src[0], b = src[1];
        x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (k + e < K) ? X[r * K + k + e] : 0.0f;
    }
    uint4 hi, lo;
    split_pair(x[0], x[1], &hi.x, &lo.x);
    split_pair(x[2], x[3], &hi.y, &lo.y);
    split_pair(x[4], x[5], &hi.z, &lo.z);
    split_pair(x[6], x[7], &hi.w, &lo.w);
    uint8_t *rec = P + ring::rec_byte(r, s, S);
    *reinterpret_cast<uint4 *>(rec + c * 16) = hi;          // hi: bytes 0 .. 31
    *reinterpret_cast<uint4 *>(rec + 32 + c * 16) = lo;     // lo: bytes 32 .. 63
}

__global__ __launch_bounds__(256) void pack_rows_kernel(const float *__restrict__ X, int64_t rows,
                                                        int64_t K, int64_t S, int vec,
                                                        uint8_t *__restrict__ P) {
    const int64_t chunks = padded_rows(rows) * S * 2;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256)
        pack_rows_chunk(X, rows, K, S, vec, P, q);
}

// Columns of X (K x cols, row-major) -> records (transposed), 64 columns x
// 64 k (4 slabs) per block through LDS: reads of X rows are contiguous
// float4s and each thread writes two half records. Columns past
// `cols` get zero records. All 256 threads must take part.
struct ColBlockRegs { float4 v[4]; };

__device__ __forceinline__ void pack_cols_load(const float *__restrict__ X, int64_t K, int64_t cols,
                                               int64_t bx, int64_t by, int vec, ColBlockRegs &r) {
    const int t = threadIdx.x;
    const int jq = (t & 15) * 4;                 // four columns 4 (t%16) .. +3
    const int64_t j = bx * 64 + jq;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t k = by * 4 * SLAB + (t >> 4) + 16 * i;
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
        r.v[i] = v;
    }
}

// Stores a loaded block to LDS, then (after a barrier) writes its records.
// The 512 half records of the block (4 slabs x 64 columns x {k 0-7, k 8-15})
// are taken two per thread; within a wave consecutive lanes take the two
// halves of consecutive records, so that each 16-byte store instruction fills
// half of every 64-byte record of two row tiles (as the row packer does),
// rather than a quarter of 64 scattered records.
__device__ __forceinline__ void pack_cols_emit(const ColBlockRegs &r, int64_t cols, int64_t S,
                                               uint8_t *__restrict__ P, int64_t bx, int64_t by,
                                               float (*tile)[64 + 4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        *reinterpret_cast<float4 *>(&tile[(t >> 4) + 16 * i][(t & 15) * 4]) = r.v[i];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int u = t + 256 * h;
        const int c = u & 1, jj = (u >> 1) & 63, part = u >> 7;
        const int64_t j = bx * 64 + jj, s = by * 4 + part;
        if (j < padded_rows(cols) && s < S) {
            const int kb = part * SLAB + c * 8;
            uint4 hi, lo;
            split_pair(tile[kb + 0][jj], tile[kb + 1][jj], &hi.x, &lo.x);
            split_pair(tile[kb + 2][jj], tile[kb + 3][jj], &hi.y, &lo.y);
            split_pair(tile[kb + 4][jj], tile[kb + 5][jj], &hi.z, &lo.z);
            split_pair(tile[kb + 6][jj], tile[kb + 7][jj], &hi.w, &lo.w);
            uint8_t *rec = P + ring::rec_byte(j, s, S);
            *reinterpret_cast<uint4 *>(rec + c * 16) = hi;          // hi: bytes 0 .. 31
            *reinterpret_cast<uint4 *>(rec + 32 + c * 16) = lo;     // lo: bytes 32 .. 63
        }
    }
    __syncthreads();                             // tile free for the next block
}

__device__ __forceinline__ void pack_cols_block(const float *__restrict__ X, int64_t K, int64_t cols,
                                                int64_t S, uint8_t *__restrict__ P, int64_t bx,
                                                int64_t by, float (*tile)[64 + 4], int vec) {
    ColBlockRegs r;
    pack_cols_load(X, K, cols, bx, by, vec, r);
    pack_cols_emit(r, cols, S, P, bx, by, tile);
}

// Each workgroup walks up to COL_BLOCKS consecutive 64-k blocks of one
// 64-column strip, loading block b+1 while it writes block b.
constexpr int COL_BLOCKS = 4;

__global__ __launch_bounds__(256) void pack_cols_kernel(const float *__restrict__ X, int64_t K,
                                                        int64_t cols, int64_t S, int vec,
                                                        uint8_t *__restrict__ P) {
    __shared__ __attribute__((aligned(16))) float tile[4 * SLAB][64 + 4];
    const int64_t by_count = (S + 3) / 4;
    const int64_t bx = blockIdx.x;
    for (int64_t by0 = (int64_t)blockIdx.y * COL_BLOCKS; by0 < by_count; by0 += (int64_t)gridDim.y * COL_BLOCKS) {
        const int64_t by_end = min(by0 + COL_BLOCKS, by_count);
        ColBlockRegs cur, next;
        pack_cols_load(X, K, cols, bx, by0, vec, cur);
        for (int64_t by = by0; by < by_end; ++by) {
            if (by + 1 < by_end) pack_cols_load(X, K, cols, bx, by + 1, vec, next);
            pack_cols_emit(cur, cols, S, P, bx, by, tile);
            cur = next;
        }
    }
}

// ---------------------------------------------------------------- stage 2 --

// Fragments of 32 records (rows) x 8 k: lane l reads row base + l%32; its hi
// values are logical chunk l/32 of the record, its lo values chunk 2 + l/32.
struct SplitMode {
    static constexpr bool SCALED = false;
    template <int FM, int FN> struct Frags { bf16x8_t ah[FM], al[FM], bh[FN], bl[FN]; };

    template <int BM, int BN, int FM, int FN>
    static __device__ __forceinline__ void read(const uint8_t *buf, int a_row, int b_row, int half,
                                                Frags<FM, FN> &f) {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            f.ah[a] = ring::lds_chunk<bf16x8_t>(buf, a_row + a * 32, half);
            f.al[a] = ring::lds_chunk<bf16x8_t>(buf, a_row + a * 32, 2 + half);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            f.bh[b] = ring::lds_chunk<bf16x8_t>(buf, b_row + b * 32, half);
            f.bl[b] = ring::lds_chunk<bf16x8_t>(buf, b_row + b * 32, 2 + half);
        }
    }

    // term-major order: consecutive matrix-core steps are independent; every
    // element sees lo.hi, hi.lo, hi.hi of each slab, slabs in ascending order
    template <int FM, int FN>
    static __device__ __forceinline__ void mma(const Frags<FM, FN> &f, f32x16_t (&acc)[FM][FN]) {
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.al[a], f.bh[b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[a], f.bl[b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[a], f.bh[b], acc[a][b], 0, 0, 0);
    }
};

ring::Operands split_operands(const uint8_t *Ap, const uint8_t *Bp, float *C, int64_t m, int64_t p,
                              int64_t S, int accumulate) {
    ring::Operands op;
    op.a0 = Ap; op.a1 = nullptr;
    op.b0 = Bp; op.b1 = nullptr;
    op.C = C;
    op.row_exp = op.col_exp = nullptr;
    op.m = m; op.p = p; op.S = S;
    op.accumulate = accumulate;
    return op;
}

// ------------------------------------------------------- grouped (persistent)
// Independent products share one launch. Members are listed longest k walk
// first; their tiles form one work list (member g owns tile ids
// [first[g], first[g+1])), and persistent workgroups claim tile ids from an
// atomic counter until the list is exhausted.
//
// Grouped members skip the conditioning pass: a tile streams the FP32 slabs
// of its rows of A and columns of B straight from memory into an LDS ring
// (direct loads, as the record ring does with records) and splits them into
// hi/lo BF16 with split_pair, as the conditioning kernels do -- either once
// per element into LDS planes (conv_tile, the default kernels) or in
// registers by every wave that reads a fragment (raw_tile). Every element of
// every member receives exactly the operation sequence of the single-product
// kernel -- the same hi/lo values, zero past n, the same matrix-core steps
// slab by slab -- so grouped and single results are bitwise equal, whichever
// kernel and block shape run.
//
// LDS stage of one slab (16 k) of raw_tile:
//   A: BM rows of 64 bytes (16 FP32), 16-byte chunk c of row r at physical
//      chunk c ^ ((r / 4) mod 4) (the record ring's swizzle);
//   B: the slab's 16 rows of BN FP32, loaded in pairs (k, k + 8) per KiB: row
//      k at bytes [0, 4 BN) of pair k mod 8, row k + 8 at [4 BN, 8 BN) rotated
//      by 128 bytes, so that the two halves of a wave (k and k + 8 of the same
//      columns) read disjoint banks.
struct GroupMember {
    const float *A, *B;
    float *C;
    int64_t m, n, p, S;
    int64_t first_tile;                 // first contraction work-list id of this member
    int32_t tiles_n, accumulate;
};

template <int BM, int BN, int WM, int WN, int NST>
struct RawCfg {
    static constexpr int WAVES_N = BN / WN, NW = (BM / WM) * WAVES_N;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int A_BYTES = BM * 64, B_BYTES = SLAB * BN * 4;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int LOADS = STAGE / 1024;            // KiB direct loads per slab
    static constexpr int LPW = LOADS / NW;
    static constexpr int LDS = NST * STAGE;
    static_assert(NW == 4 && BN == 128 && BM % 16 == 0 && LOADS % NW == 0, "shape of the raw ring");
};

// 8 FP32 values -> hi and lo BF16 fragments
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8_t &hi, bf16x8_t &lo) {
    uint4 h, l;
    split_pair(x[0], x[1], &h.x, &l.x);
    split_pair(x[2], x[3], &h.y, &l.y);
    split_pair(x[4], x[5], &h.z, &l.z);
    split_pair(x[6], x[7], &h.w, &l.w);
    hi = __builtin_bit_cast(bf16x8_t, h);
    lo = __builtin_bit_cast(bf16x8_t, l);
}

// A wave's FM x FN blocks of 32 x 32 accumulators to C (rows from i0,
// columns from j0), skipping what lies past m or p. The accumulate form
// (ACC) reads a block's 16 values of C before any store, so the loads are in
// flight together; the overwrite form has no trace of it.
template <bool ACC, int FM, int FN>
__device__ __forceinline__ void store_blocks(const GroupMember &d, int64_t i0, int64_t j0,
                                             const f32x16_t (&acc)[FM][FN]) {
    const int lane = threadIdx.x & 63;
    const int64_t p = d.p;
    ring::global_f32 *C = (ring::global_f32 *)d.C;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t j = j0 + b * 32 + (lane & 31);
            if (j >= p) continue;
            float old[16];
            if constexpr (ACC) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t i = i0 + a * 32 + mfma32_row(r, lane);
                    if (i < d.m) old[r] = C[i * p + j];
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + a * 32 + mfma32_row(r, lane);
                if (i < d.m) {
                    float v = acc[a][b][r];
                    if constexpr (ACC) v += old[r];
                    C[i * p + j] = v;
                }
            }
        }
}

template <int FM, int FN>
__device__ __forceinline__ void store_block(const GroupMember &d, int64_t i0, int64_t j0,
                                            const f32x16_t (&acc)[FM][FN]) {
    if (d.accumulate)
        store_blocks<true, FM, FN>(d, i0, j0, acc);
    else
        store_blocks<false, FM, FN>(d, i0, j0, acc);
}

template <int BM, int BN, int WM, int WN, int NST>
__device__ __forceinline__ void raw_tile(const GroupMember &d, int64_t i0, int64_t j0, uint8_t *lds) {
    using G = RawCfg<BM, BN, WM, WN, NST>;
    constexpr int FM = G::FM, FN = G::FN, STAGE = G::STAGE, LPW = G::LPW;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave / G::WAVES_N, wn = wave % G::WAVES_N;
    const int L = (int)d.S;
    const int64_t n = d.n, p = d.p;

    // Both resources start at the slab (A: column k0 of the tile's first row,
    // B: row k0) and end where the live data ends, so each lane's vector
    // offset is the same for every slab (computed once, in registers that no
    // later instruction overwrites). Rows past m and k past the last live
    // row's end are out of range (zeros); k past n inside earlier rows reads
    // the next row and is masked when split.
    const int64_t rows_live = d.m - i0 < BM ? d.m - i0 : BM;
    const int64_t a_range = rows_live * n * 4;
    const float *a_tile = d.A + i0 * n;
    const float *b_tile = d.B + j0;
    const int64_t b_total = n * p - j0;                  // elements from b_tile to the end of B
    int voff[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int g = wave * LPW + q;                    // wave-uniform load index
        if (g < BM / 16) {
            const int r = 16 * g + (lane >> 2);
            const int c = (lane & 3) ^ ((lane >> 4) & 3);
            voff[q] = r < rows_live ? (int)(((int64_t)r * n + 4 * c) * 4) : ring::kDeadVoffset;
        } else {
            const int h = g - BM / 16;                   // pair h: rows h and h + 8 of the slab
            const int upper = lane >> 5;
            const int gc = upper ? ((lane & 31) + 8) & 31 : lane & 31;
            voff[q] = (int)(((int64_t)(h + 8 * upper) * p + 4 * gc) * 4);
        }
    }

    auto issue_to = [&](uint8_t *buf, int s) {         // buf: stage s mod NST
        const int64_t k0 = (int64_t)s * SLAB;
        const int64_t a_left = a_range - k0 * 4, b_left = (b_total - k0 * p) * 4;
        const __amdgpu_buffer_rsrc_t a_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a_tile + k0), (short)0, (int)(a_left > 0 ? a_left : 0), 0x00020000);
        const __amdgpu_buffer_rsrc_t b_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(b_tile + k0 * p), (short)0,
            (int)(b_left < 0x7FFFFFFF ? (b_left > 0 ? b_left : 0) : 0x7FFFFFFF), 0x00020000);
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int g = wave * LPW + q;
            if (g < BM / 16)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(a_rsrc, (ring::lds_void_t *)(buf + g * 1024), 16, voff[q],
                                                         0, 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(b_rsrc,
                                                         (ring::lds_void_t *)(buf + G::A_BYTES + (g - BM / 16) * 1024),
                                                         16, voff[q], 0, 0, 0);
        }
    };

    const int frow = lane & 31, fhalf = lane >> 5;
    float ra[FM][8], rb[FN][8];
    // raw fragments of a slab (in buf): A rows (8 k of half fhalf), B columns (8 k rows)
    auto read_raw_from = [&](const uint8_t *buf) {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            const int r = wm * WM + a * 32 + frow;
            const int sw = (r >> 2) & 3;
            const float4 lo4 = *reinterpret_cast<const float4 *>(buf + r * 64 + (((2 * fhalf) ^ sw) << 4));
            const float4 hi4 = *reinterpret_cast<const float4 *>(buf + r * 64 + (((2 * fhalf + 1) ^ sw) << 4));
            ra[a][0] = lo4.x; ra[a][1] = lo4.y; ra[a][2] = lo4.z; ra[a][3] = lo4.w;
            ra[a][4] = hi4.x; ra[a][5] = hi4.y; ra[a][6] = hi4.z; ra[a][7] = hi4.w;
        }
        const uint8_t *bb = buf + G::A_BYTES;
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int cb = wn * WN + b * 32 + frow;
            const int off = fhalf ? 512 + ((((cb >> 2) + 24) & 31) << 4) + ((cb & 3) << 2) : cb << 2;
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[b][e] = *reinterpret_cast<const float *>(bb + e * 1024 + off);
        }
    };
    SplitMode::Frags<FM, FN> f;
    // split into fragments; k past n (the last slab) counts as zero
    auto convert = [&](int s) {
        const int64_t kb = (int64_t)s * SLAB + 8 * fhalf;
        if (kb + 8 > n) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (kb + e >= n) {
#pragma unroll
                    for (int a = 0; a < FM; ++a) ra[a][e] = 0.0f;
#pragma unroll
                    for (int b = 0; b < FN; ++b) rb[b][e] = 0.0f;
                }
        }
#pragma unroll
        for (int a = 0; a < FM; ++a) split8(ra[a], f.ah[a], f.al[a]);
#pragma unroll
        for (int b = 0; b < FN; ++b) split8(rb[b], f.bh[b], f.bl[b]);
    };

    f32x16_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16_t{};

    auto wait_loads = [&](int stages) {
        switch (stages <= 0 ? 0 : stages >= 2 ? 2 : stages) {
        case 0: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(0)); break;
        case 1: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(LPW)); break;
        default: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(2 * LPW)); break;
        }
    };
    static_assert(NST >= 3 && NST <= 4, "up to two slabs in flight");

    // the loads of a step fill one stage while the fragments of the next
    // slab are read from another: disjoint LDS, passed as restrict pointers
    // so that the reads need not wait for those loads
    auto step = [&](uint8_t *__restrict__ dma, const uint8_t *__restrict__ src, int s) {
        if (s + NST - 1 < L) issue_to(dma, s + NST - 1);
        read_raw_from(src);
    };
    if (L > 0) {
        for (int q = 0; q < NST - 1; ++q)
            if (q < L) issue_to(lds + q * STAGE, q);
        wait_loads(min(NST - 2, L - 1));
        ring::ring_barrier();
        read_raw_from(lds);
        convert(0);
        for (int s = 0; s < L; ++s) {
            if (s + 1 < L) {
                // slab s + 1 landed in every wave; the buffer of slab s - 1 is free
                wait_loads(min(NST - 3, L - s - 2));
                ring::ring_barrier();
                step(lds + ((s + NST - 1) % NST) * STAGE, lds + ((s + 1) % NST) * STAGE, s);
            }
            SplitMode::mma<FM, FN>(f, acc);
            if (s + 1 < L) convert(s + 1);
        }
    }
    __syncthreads();                    // every wave done with the ring before the next tile's loads
    store_block<FM, FN>(d, i0 + wm * WM, j0 + wn * WN, acc);
}

// Work-list claims, XCD by XCD. The tile list is cut into eight segments of
// about equal work, one per XCD (workgroups go to the XCDs round-robin by id),
// each a run of whole members, so that the tiles sharing a member's rows and
// columns run under one L2. A workgroup claims from its own XCD's segment
// (counter 4 x, bounds[x] .. bounds[x + 1]) and, once that is drained, from
// the next XCDs' in turn; `seg` counts the segments it found drained. Called
// by one thread; -1: nothing left anywhere.
__device__ __forceinline__ int64_t claim_tile(unsigned long long *ctr, const int64_t *bounds, int &seg) {
    const int xcd = blockIdx.x & 7;
    while (seg < 8) {
        const int x = (xcd + seg) & 7;
        const int64_t t = bounds[x] + (int64_t)atomicAdd(ctr + 4 * x, 1ull);
        if (t < bounds[x + 1]) return t;
        ++seg;
    }
    return -1;
}

template <int BM, int BN, int WM, int WN, int NST>
__global__ __launch_bounds__(256, 2) void split_grouped_kernel(const GroupMember *__restrict__ g,
                                                               const int32_t *__restrict__ tile_owner,
                                                               const int64_t *__restrict__ bounds,
                                                               unsigned long long *__restrict__ counter) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[RawCfg<BM, BN, WM, WN, NST>::LDS];
    __shared__ int64_t s_tile;
    int seg = 0;
    for (;;) {
        __syncthreads();                // nobody still reads s_tile
        if (threadIdx.x == 0) s_tile = claim_tile(counter, bounds, seg);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile < 0) break;
        const int k = __builtin_amdgcn_readfirstlane(tile_owner[tile]);
        const GroupMember &d = g[k];
        const int64_t local = tile - d.first_tile;
        const int64_t tm = local / d.tiles_n, tn = local - tm * d.tiles_n;
        raw_tile<BM, BN, WM, WN, NST>(d, __builtin_amdgcn_readfirstlane((int)tm) * (int64_t)BM,
                                      __builtin_amdgcn_readfirstlane((int)tn) * (int64_t)BN, lds);
    }
}

// Grouped block that splits every element of a slab once. The FP32 slab
// lands in an LDS ring by direct loads as above (A swizzled; B as plain rows
// of BN FP32); one pass of the whole workgroup turns it into hi and lo BF16
// planes in a second, double-buffered LDS area; the four waves (2 x 2, each
// BM/2 x BN/2) read their matrix-core fragments straight from the planes.
// Per slab and wave this costs a quarter of the splits of the raw ring (no
// element is split by two waves) and one barrier, which at once publishes
// the planes just written, confirms the next raw slab landed in every wave
// and frees the raw stage just split for the next load.
//
// Plane layout, per plane (A hi, A lo, B hi, B lo): [half h][row or column]
// [8 BF16 of k in 8h .. 8h + 7], i.e. 16 bytes per row and half, so that a
// fragment (32 rows, two halves) is two runs of 512 contiguous bytes.
template <int BM, int BN, int NST, int NCV> struct ConvCfg {
    static constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
    static constexpr int RAW_A = BM * 64, RAW_B = SLAB * BN * 4, RAW = RAW_A + RAW_B;
    static constexpr int PL_A = BM * 32, PL_B = BN * 32;       // bytes of one A or B plane
    static constexpr int CONV = 2 * (PL_A + PL_B);
    static constexpr int LOADS = RAW / 1024, LPW = LOADS / 4;  // KiB direct loads per slab, per wave
    static constexpr int UNITS = 2 * (BM + BN);                // half rows of A, half columns of B
    static constexpr int LDS = NST * RAW + NCV * CONV;
    static_assert((BM == 64 || BM == 128) && (BN == 64 || BN == 128), "blocks of the split-once ring");
    static_assert(LOADS % 4 == 0 && NST >= 2 && NST <= 4 && (NCV == 1 || NCV == 2), "shape of the split-once ring");
};

template <int BM, int BN, int NST, int NCV>
__device__ __forceinline__ void conv_tile(const GroupMember &d, int64_t i0, int64_t j0, uint8_t *lds) {
    using G = ConvCfg<BM, BN, NST, NCV>;
    constexpr int FM = G::FM, FN = G::FN, LPW = G::LPW;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int L = (int)d.S;
    const int64_t n = d.n, p = d.p;
    uint8_t *const raw = lds;
    uint8_t *const conv = lds + NST * G::RAW;

    const int64_t rows_live = d.m - i0 < BM ? d.m - i0 : BM;
    const int64_t a_range = rows_live * n * 4;
    const float *a_tile = d.A + i0 * n;
    const float *b_tile = d.B + j0;
    const int64_t b_total = n * p - j0;                  // elements from b_tile to the end of B

    // Slab s into raw stage s mod NST. Both resources start at the slab (A:
    // column k0 of the tile's first row; B: row k0) and end where the live
    // data ends, so the lanes' vector offsets stay the same for every slab --
    // computed once here, in registers that no later instruction overwrites
    // (a register the direct loads still read would make the compiler wait for
    // every load in flight before reusing it). A: 16 rows of 64 bytes per
    // load, rows past m dead, k past n in the last live row out of range
    // (zeros), k past n inside earlier rows reads the next row (masked when
    // split). B: 1024 / (4 BN) rows per load; rows past n (and columns past p
    // on the last row) are out of range and load as zeros.
    int voff[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int g = wave * LPW + q;
        if (g < BM / 16) {
            const int r = 16 * g + (lane >> 2);
            const int c = (lane & 3) ^ ((lane >> 4) & 3);
            voff[q] = r < rows_live ? (int)(((int64_t)r * n + 4 * c) * 4) : ring::kDeadVoffset;
        } else {
            constexpr int CPR = BN / 4;                     // 16-byte chunks per B row
            const int row = (g - BM / 16) * (1024 / (4 * BN)) + lane / CPR;
            voff[q] = (int)(((int64_t)row * p + 4 * (lane % CPR)) * 4);
        }
    }
    auto issue_to = [&](uint8_t *buf, int s) {       // buf: raw stage s mod NST
        const int64_t k0 = (int64_t)s * SLAB;
        const int64_t a_left = a_range - k0 * 4, b_left = (b_total - k0 * p) * 4;
        const __amdgpu_buffer_rsrc_t a_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a_tile + k0), (short)0, (int)(a_left > 0 ? a_left : 0), 0x00020000);
        const __amdgpu_buffer_rsrc_t b_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(b_tile + k0 * p), (short)0,
            (int)(b_left < 0x7FFFFFFF ? (b_left > 0 ? b_left : 0) : 0x7FFFFFFF), 0x00020000);
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int g = wave * LPW + q;
            if (g < BM / 16)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(a_rsrc, (ring::lds_void_t *)(buf + g * 1024), 16, voff[q],
                                                         0, 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(b_rsrc,
                                                         (ring::lds_void_t *)(buf + G::RAW_A + (g - BM / 16) * 1024),
                                                         16, voff[q], 0, 0, 0);
        }
    };

    // Split raw slab s (in buf) into the plane set cv; k past n counts as zero.
    auto convert_from = [&](const uint8_t *buf, uint8_t *cv, int s) {
        const int64_t k0 = (int64_t)s * SLAB;
#pragma unroll
        for (int i = 0; i < (G::UNITS + 255) / 256; ++i) {
            const int ub = wave * 64 + 256 * i;     // first unit of this wave: units split per wave
            if (ub >= G::UNITS) break;
            const int u = ub + lane;
            float x[8];
            int h, dst;
            const bool is_a = ub < 2 * BM;
            if (is_a) {
                h = ub / BM;
                const int r = u - h * BM;
                const int sw = (r >> 2) & 3;
                const float4 v0 = *reinterpret_cast<const float4 *>(buf + r * 64 + (((2 * h) ^ sw) << 4));
                const float4 v1 = *reinterpret_cast<const float4 *>(buf + r * 64 + (((2 * h + 1) ^ sw) << 4));
                x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
                x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
                dst = h * BM * 16 + r * 16;
            } else {
                h = (ub - 2 * BM) / BN;
                const int c = u - 2 * BM - h * BN;
                const uint8_t *bb = buf + G::RAW_A + c * 4;
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = *reinterpret_cast<const float *>(bb + (8 * h + e) * BN * 4);
                dst = 2 * G::PL_A + h * BN * 16 + c * 16;
            }
            if (k0 + SLAB > n) {
                const int live = (int)(n - k0) - 8 * h;     // live k of this unit's 8 (can be <= 0)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (e >= live) x[e] = 0.0f;
            }
            bf16x8_t hi, lo;
            split8(x, hi, lo);
            const int plane = is_a ? G::PL_A : G::PL_B;
            *reinterpret_cast<bf16x8_t *>(cv + dst) = hi;
            *reinterpret_cast<bf16x8_t *>(cv + dst + plane) = lo;
        }
    };

    const int frow = lane & 31, fhalf = lane >> 5;
    SplitMode::Frags<FM, FN> f;
    auto read_frags_from = [&](const uint8_t *cv) {
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            const int off = fhalf * BM * 16 + (wm * G::WM + a * 32 + frow) * 16;
            f.ah[a] = *reinterpret_cast<const bf16x8_t *>(cv + off);
            f.al[a] = *reinterpret_cast<const bf16x8_t *>(cv + G::PL_A + off);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int off = 2 * G::PL_A + fhalf * BN * 16 + (wn * G::WN + b * 32 + frow) * 16;
            f.bh[b] = *reinterpret_cast<const bf16x8_t *>(cv + off);
            f.bl[b] = *reinterpret_cast<const bf16x8_t *>(cv + G::PL_B + off);
        }
    };

    f32x16_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16_t{};

    auto wait_loads = [&](int slabs) {          // at most `slabs` later slabs of this wave in flight
        switch (slabs <= 0 ? 0 : slabs >= 3 ? 3 : slabs) {
        case 0: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(0)); break;
        case 1: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(LPW)); break;
        case 2: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(2 * LPW)); break;
        default: __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(3 * LPW)); break;
        }
    };
    static_assert(3 * LPW <= 63, "vmcnt counts up to 63 operations");
    // Barrier that also publishes this wave's plane writes (LDS stores done).
    auto plane_barrier = [] {
        __builtin_amdgcn_s_waitcnt(0xC07F);     // lgkmcnt(0); vector-memory and export counts not waited on
        ring::ring_barrier();
    };

    // One slab step. The stage the step's direct loads fill (dma: raw stage
    // s mod NST, split by every wave before this step), the stage it splits
    // (src: slab s + 1) and the plane sets are disjoint LDS, passed as
    // restrict pointers: that lets the compiler see that reading src or the
    // planes need not wait for the loads into dma, which are meant to stay in
    // flight (the explicit waits above order each slab's loads before its
    // split).
    // The matrix-core steps of slab s are issued as soon as its fragments are
    // in registers, before the split of slab s + 1, so that they run while
    // this wave splits; the wave issues them at raised priority, so that the
    // other workgroups' split work does not hold them back.
    auto mma_step = [&] {
        __builtin_amdgcn_s_setprio(1);
        SplitMode::mma<FM, FN>(f, acc);
        __builtin_amdgcn_s_setprio(0);
    };
    auto step1 = [&](uint8_t *__restrict__ dma, const uint8_t *__restrict__ src, uint8_t *__restrict__ planes,
                     int s) {
        // one plane set: a second barrier between reading it and overwriting
        // it with the next slab
        if (s + NST < L) issue_to(dma, s + NST);
        read_frags_from(planes);
        mma_step();
        if (s + 1 < L) {
            wait_loads((NST - 1 < L - 2 - s) ? NST - 1 : L - 2 - s);
            plane_barrier();
            convert_from(src, planes, s + 1);
        }
    };
    auto step2 = [&](uint8_t *__restrict__ dma, const uint8_t *__restrict__ src,
                     const uint8_t *__restrict__ planes_r, uint8_t *__restrict__ planes_w, int s) {
        // two plane sets: one barrier makes the planes of s complete, raw
        // slab s + 1 landed and the planes of s - 1 (the set this step
        // writes) read by every wave
        if (s + 1 < L) wait_loads((NST - 2 < L - 2 - s) ? NST - 2 : L - 2 - s);
        plane_barrier();
        if (s + NST < L) issue_to(dma, s + NST);
        read_frags_from(planes_r);
        mma_step();
        if (s + 1 < L) convert_from(src, planes_w, s + 1);
    };

    // Ring fill and the split of slab 0 (stage 0), while the later stages'
    // loads stay in flight (disjoint: restrict, as in the steps).
    auto prologue = [&](uint8_t *__restrict__ st0, uint8_t *__restrict__ later, uint8_t *__restrict__ planes) {
        issue_to(st0, 0);
        for (int q = 1; q < NST; ++q)
            if (q < L) issue_to(later + (q - 1) * G::RAW, q);
        wait_loads((NST < L ? NST : L) - 1);
        ring::ring_barrier();
        convert_from(st0, planes, 0);
    };

    if (L > 0) {
        prologue(raw, raw + G::RAW, conv);
        for (int s = 0; s < L; ++s) {
            uint8_t *dma = raw + (s % NST) * G::RAW;
            const uint8_t *src = raw + ((s + 1) % NST) * G::RAW;
            if (NCV == 2) {
                step2(dma, src, conv + (s & 1) * G::CONV, conv + ((s + 1) & 1) * G::CONV, s);
            } else {
                plane_barrier();
                step1(dma, src, conv, s);
            }
        }
    }
    __syncthreads();                    // every wave done with both LDS areas before the next tile
    store_block<FM, FN>(d, i0 + wm * G::WM, j0 + wn * G::WN, acc);
}

template <int BM, int BN, int NST, int NCV, int OCC>
__global__ __launch_bounds__(256, OCC) void split_grouped_conv_kernel(const GroupMember *__restrict__ g,
                                                                    const int32_t *__restrict__ tile_owner,
                                                                    const int64_t *__restrict__ bounds,
                                                                    unsigned long long *__restrict__ counter) {
    using G = ConvCfg<BM, BN, NST, NCV>;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[G::LDS];
    // the claimed tile id lives in the last plane set, which no wave writes
    // before the first barrier of a tile
    int64_t *s_tile = reinterpret_cast<int64_t *>(lds + NST * G::RAW + (NCV - 1) * G::CONV);
    int seg = 0;
    for (;;) {
        __syncthreads();                // nobody still reads the tile id (or the planes)
        if (threadIdx.x == 0) *s_tile = claim_tile(counter, bounds, seg);
        __syncthreads();
        const int64_t tile = *s_tile;
        if (tile < 0) break;
        const int k = __builtin_amdgcn_readfirstlane(tile_owner[tile]);
        const GroupMember &d = g[k];
        const int64_t local = tile - d.first_tile;
        const int64_t tm = local / d.tiles_n, tn = local - tm * d.tiles_n;
        conv_tile<BM, BN, NST, NCV>(d, __builtin_amdgcn_readfirstlane((int)tm) * (int64_t)BM,
                               __builtin_amdgcn_readfirstlane((int)tn) * (int64_t)BN, lds);
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

struct SplitShape { int bm, bn, wm, wn, stages; };
// (deeper rings were measured no faster for this path at N = 8192). The
// rectangular blocks run four waves of 128 x 64 or 64 x 128, two workgroups
// per CU.
constexpr SplitShape kSplit[] = {{128, 128, 64, 64, 3}, {256, 256, 128, 64, 3}, {256, 128, 128, 64, 3},
                                 {128, 256, 64, 128, 3}};

template <int BM, int BN, int WM, int WN, int NST>
hipError_t launch_shape(const moa_gemm_desc &d, const uint8_t *Ap, const uint8_t *Bp, int64_t S,
                        hipStream_t st) {
    const ring::Operands op = split_operands(Ap, Bp, static_cast<float *>(d.C), d.m, d.p, S, d.accumulate);
    const int tiles_m = (int)((d.m + BM - 1) / BM);
    const int tiles_n = (int)((d.p + BN - 1) / BN);
    hipLaunchKernelGGL((ring::single_kernel<BM, BN, WM, WN, 1, SplitMode, NST>), dim3(tiles_m * tiles_n),
                       dim3(ring::Cfg<BM, BN, WM, WN, 1, NST>::THREADS), 0, st, op, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace

int split_bf16_variant_count() { return (int)(sizeof(kSplit) / sizeof(kSplit[0])); }

// Default block: 256 x 256 (one workgroup per CU) once it gives every CU a
// block, else 128 x 128. When its blocks fill more than one round of the CUs
// but leave the last round less than 40% full, the rectangular blocks (two
// per CU, half the area) shorten that tail: measured N = 6144 and 7168
// (2.25 and 3.06 rounds) 7-9% faster, while 256 x 256 stays ahead at whole
// or well-filled rounds (N = 4096, 5120, 8192, 12288).
int split_bf16_default_variant(int64_t m, int64_t p) {
    const int64_t big = ((m + 255) / 256) * ((p + 255) / 256);
    if (big < kNumCUs) return 0;
    const int64_t tail = big % kNumCUs;
    if (big > kNumCUs && tail != 0 && 10 * tail < 4 * kNumCUs) return p >= m ? 3 : 2;
    return 1;
}

int64_t split_bf16_workspace_bytes(int64_t m, int64_t n, int64_t p) {
    const int64_t S = (n + SLAB - 1) / SLAB;
    return ring::array_bytes(m, S) + ring::array_bytes(p, S);
}

void split_bf16_shape(int v, Plan *p) {
    const SplitShape s = kSplit[v];
    p->variant = v;
    p->tile_m = s.bm;
    p->tile_n = s.bn;
    p->tile_k = SLAB;
    p->wave_m = s.wm;
    p->wave_n = s.wn;
    p->lane_m = p->lane_n = 0;
    p->threads = (s.bm / s.wm) * (s.bn / s.wn) * 64;
    p->lds_bytes = s.stages * (s.bm + s.bn) * REC_BYTES;
}

namespace {
// Records of the `rows` rows of a row-major rows x K array.
void rows_records(const float *X, int64_t rows, int64_t K, int64_t S, uint8_t *P, hipStream_t st) {
    const int vec = (K % 8 == 0) && ((uintptr_t)X % 16 == 0);
    int64_t blocks = (padded_rows(rows) * S * 2 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, K, S, vec, P);
}
// Records of the `cols` columns of a row-major K x cols array.
void cols_records(const float *X, int64_t K, int64_t cols, int64_t S, uint8_t *P, hipStream_t st) {
    const int vec = (cols % 4 == 0) && ((uintptr_t)X % 16 == 0);
    const int64_t by = ((S + 3) / 4 + COL_BLOCKS - 1) / COL_BLOCKS;
    hipLaunchKernelGGL(pack_cols_kernel, dim3((unsigned)((cols + 63) / 64), (unsigned)(by < 65535 ? by : 65535)),
                       dim3(256), 0, st, X, K, cols, S, vec, P);
}
}  // namespace

// Records of A's rows and B's columns. A column-major A (element (i, k) at
// i + k m) is a row-major n x m array whose columns are A's rows; a
// column-major B is a row-major p x n array whose rows are B's columns.
hipError_t launch_split_pack(const moa_gemm_desc &d, void *ws, hipStream_t st) {
    const int64_t S = (d.n + SLAB - 1) / SLAB;
    uint8_t *Ap = static_cast<uint8_t *>(ws);
    uint8_t *Bp = Ap + ring::array_bytes(d.m, S);
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    if (S == 0) return hipSuccess;
    if (d.flags & MOA_FLAG_A_COL) cols_records(A, d.n, d.m, S, Ap, st);
    else rows_records(A, d.m, d.n, S, Ap, st);
    if (d.flags & MOA_FLAG_B_COL) rows_records(B, d.p, d.n, S, Bp, st);
    else cols_records(B, d.n, d.p, S, Bp, st);
    return hipGetLastError();
}

hipError_t launch_split_bf16(const moa_gemm_desc &d, const Plan &plan, void *ws, hipStream_t st) {
    hipError_t e;
    {
        TraceScope ts(MOA_K_SPLIT_PACK, st);
        e = launch_split_pack(d, ws, st);
    }
    if (e != hipSuccess) return e;
    TraceScope ts(MOA_K_SPLIT_BF16, st);
    const int64_t S = (d.n + SLAB - 1) / SLAB;
    const uint8_t *Ap = static_cast<const uint8_t *>(ws);
    const uint8_t *Bp = Ap + ring::array_bytes(d.m, S);
    if (plan.split_k > 1) {
        const ring::Operands op = split_operands(Ap, Bp, static_cast<float *>(d.C), d.m, d.p, S, d.accumulate);
        float *partials = reinterpret_cast<float *>(static_cast<char *>(ws) + plan.partial_offset);
        return ring::launch_splitk<128, 128, 64, 64, 1, SplitMode, 3>(op, plan.split_k, partials, st);
    }
    switch (plan.variant) {
    case 0: return launch_shape<128, 128, 64, 64, 3>(d, Ap, Bp, S, st);
    case 2: return launch_shape<256, 128, 128, 64, 3>(d, Ap, Bp, S, st);
    case 3: return launch_shape<128, 256, 64, 128, 3>(d, Ap, Bp, S, st);
    default: return launch_shape<256, 256, 128, 64, 3>(d, Ap, Bp, S, st);
    }
}

namespace {
__global__ void zero_counters_kernel(unsigned long long *x) {
    if (threadIdx.x < 8) x[4 * threadIdx.x] = 0ull;
}
constexpr int GB_M = 128, GW_M = 64, GW_N = 64, G_NST = 4;   // largest grouped block rows; raw-ring waves, depth

// Persistent kernels of a grouped launch: block, workgroups per CU, and the
// relative time of one slab step of a block (measured on 256 x n x 256
// members), which the static rule weighs slab steps with.
struct GroupedKernel { int bm, bn, occ; double step_cost; };
constexpr GroupedKernel kGroupedK[] = {
    {128, 128, 3, 1.00},   // 0: split once into one plane set, two raw stages
    {128, 128, 2, 1.25},   // 1: split once, two plane sets, three raw stages
    {128, 128, 2, 0.95},   // 2: split in registers by every wave that reads a fragment
    {64, 128, 4, 0.75},    // 3: split once, 64 x 128
    {128, 64, 4, 0.75},    // 4: split once, 128 x 64
};
constexpr int kGroupedVariants = (int)(sizeof(kGroupedK) / sizeof(kGroupedK[0]));
int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

int64_t member_tiles(const moa_gemm_desc &d, int bm, int bn) {
    return ((d.m + bm - 1) / bm) * ((d.p + bn - 1) / bn);
}

// Contraction tiles of a member list under any variant (64 x 64 blocks: at
// least as many as every block of the table), for sizing the tables.
GroupedWork grouped_counts(const moa_gemm_desc *const *members, int count) {
    GroupedWork w{0, 0, 0};
    for (int k = 0; k < count; ++k) w.tiles += member_tiles(*members[k], 64, 64);
    return w;
}
// Member table, then the nine segment bounds of the XCD claims (int64, 256
// bytes), then the tile -> member table (int32): the part a launch uses is
// one prefix of the table.
int64_t members_bytes(int count) { return align256((int64_t)count * (int64_t)sizeof(GroupMember)); }
int64_t table_bytes(int count, const GroupedWork &w) { return members_bytes(count) + 256 + align256(4 * w.tiles); }
}  // namespace

// The raw ring addresses a tile's rows of A with 32-bit offsets (128 rows of
// n FP32) and a slab of B likewise (16 rows of p FP32).
bool split_grouped_fits(const moa_gemm_desc &d) {
    return ((int64_t)GB_M + 1) * d.n * 4 < 0x7FFFFFFF && ((int64_t)SLAB + 1) * d.p * 4 < 0x7FFFFFFF;
}

int64_t split_grouped_desc_bytes(const moa_gemm_desc *const *members, int count) {
    return table_bytes(count, grouped_counts(members, count));
}

int64_t split_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count) {
    return 256 + split_grouped_desc_bytes(members, count);
}

int split_grouped_variant_count() { return kGroupedVariants; }

// Static rule: the block with the fewest weighted slab steps over the
// members (ties to the earlier variant in the list); variants 0 and 1 are
// left to the autotuner (variant 2 measured 1-12% faster than variant 0 on
// the batching workload and 10-15% on groups of 1024^3 and 2048^3 products,
// the same on groups of small ones).
int split_grouped_default_variant(const moa_gemm_desc *const *members, int count) {
    int best = 2;
    double best_cost = 0;
    for (int v : {2, 3, 4}) {
        double cost = 0;
        for (int k = 0; k < count; ++k) {
            const moa_gemm_desc &d = *members[k];
            cost += (double)member_tiles(d, kGroupedK[v].bm, kGroupedK[v].bn) * (double)((d.n + SLAB - 1) / SLAB);
        }
        cost *= kGroupedK[v].step_cost;
        if (v == 2 || cost < best_cost) {
            best = v;
            best_cost = cost;
        }
    }
    return best;
}

// Lays out the members in `host_staging` for grouped kernel `variant`;
// returns the tile count. Members are dealt, heaviest first (tiles x slab
// steps), to the lightest of eight XCD segments; inside a segment they run
// longest k walk first, so each segment's tail holds its cheapest tiles. The
// device member array is at ws + 256, the claim counters at ws.
GroupedWork split_grouped_layout(const moa_gemm_desc *const *members, int count, void *ws,
                                 void *host_staging, int variant) {
    (void)ws;
    const GroupedKernel gk = kGroupedK[variant];
    auto cost = [&](int k) {
        const moa_gemm_desc &d = *members[k];
        return (double)member_tiles(d, gk.bm, gk.bn) * (double)((d.n + SLAB - 1) / SLAB);
    };
    std::vector<int> heavy(count);
    for (int k = 0; k < count; ++k) heavy[k] = k;
    std::stable_sort(heavy.begin(), heavy.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<int> seg_of(count);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k : heavy) {
        int x = 0;
        for (int y = 1; y < 8; ++y)
            if (load[y] < load[x]) x = y;
        seg_of[k] = x;
        load[x] += cost(k);
    }
    std::vector<int> order(count);
    for (int k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (seg_of[a] != seg_of[b]) return seg_of[a] < seg_of[b];
        return members[a]->n > members[b]->n;
    });
    char *base = static_cast<char *>(host_staging);
    GroupMember *h = reinterpret_cast<GroupMember *>(base);
    int32_t *tile_owner = reinterpret_cast<int32_t *>(base + members_bytes(count) + 256);
    int64_t tiles = 0;
    int64_t bounds[9];
    int next_seg = 0;
    for (int q = 0; q < count; ++q) {
        const moa_gemm_desc &d = *members[order[q]];
        while (next_seg <= seg_of[order[q]]) bounds[next_seg++] = tiles;
        GroupMember g{};
        g.A = static_cast<const float *>(d.A);
        g.B = static_cast<const float *>(d.B);
        g.C = static_cast<float *>(d.C);
        g.m = d.m; g.n = d.n; g.p = d.p;
        g.S = (d.n + SLAB - 1) / SLAB;
        g.first_tile = tiles;
        g.tiles_n = (int32_t)((d.p + gk.bn - 1) / gk.bn);
        g.accumulate = d.accumulate;
        const int64_t mt = ((d.m + gk.bm - 1) / gk.bm) * g.tiles_n;
        for (int64_t t = 0; t < mt; ++t) tile_owner[tiles + t] = q;
        tiles += mt;
        h[q] = g;
    }
    while (next_seg <= 8) bounds[next_seg++] = tiles;
    std::memcpy(base + members_bytes(count), bounds, sizeof(bounds));
    return {tiles, 0, variant, members_bytes(count) + 256 + 4 * tiles};
}

namespace {
// The persistent contraction of a grouped launch whose member table and
// cleared claim counters are in place.
hipError_t launch_persistent(void *ws, int count, const GroupedWork &work, hipStream_t st) {
    const int64_t tiles = work.tiles;
    char *base = static_cast<char *>(ws);
    unsigned long long *counter = reinterpret_cast<unsigned long long *>(base);
    const GroupMember *dev_members = reinterpret_cast<const GroupMember *>(base + 256);
    const int64_t *bounds = reinterpret_cast<const int64_t *>(base + 256 + members_bytes(count));
    const int32_t *tile_owner = reinterpret_cast<const int32_t *>(base + 256 + members_bytes(count) + 256);
    const int v = work.variant;
    const int64_t grid = std::min<int64_t>(tiles, (int64_t)kGroupedK[v].occ * kNumCUs);   // resident blocks
    TraceScope ts(MOA_K_SPLIT_GROUPED, st);
    if (grid <= 0) return hipGetLastError();
    const dim3 gr((unsigned)grid), bl(256);
    switch (v) {
    case 1:
        hipLaunchKernelGGL((split_grouped_conv_kernel<128, 128, 3, 2, 2>), gr, bl, 0, st, dev_members, tile_owner,
                           bounds, counter);
        break;
    case 2:
        hipLaunchKernelGGL((split_grouped_kernel<128, 128, GW_M, GW_N, G_NST>), gr, bl, 0, st, dev_members,
                           tile_owner, bounds, counter);
        break;
    case 3:
        hipLaunchKernelGGL((split_grouped_conv_kernel<64, 128, 2, 1, 4>), gr, bl, 0, st, dev_members, tile_owner,
                           bounds, counter);
        break;
    case 4:
        hipLaunchKernelGGL((split_grouped_conv_kernel<128, 64, 2, 1, 4>), gr, bl, 0, st, dev_members, tile_owner,
                           bounds, counter);
        break;
    default:
        hipLaunchKernelGGL((split_grouped_conv_kernel<128, 128, 2, 1, 3>), gr, bl, 0, st, dev_members, tile_owner,
                           bounds, counter);
        break;
    }
    return hipGetLastError();
}

// Uploads the used prefix of a member table (n16 16-byte words) straight from
// pinned host memory mapped into the device's address space, and clears the
// claim counters: one small kernel in place of a copy-engine transfer, whose
// hand-offs to and from the compute queue cost more than the copy.
__global__ __launch_bounds__(256) void stage_table_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          int64_t n16, unsigned long long *__restrict__ counters) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0 && threadIdx.x < 8) counters[4 * threadIdx.x] = 0ull;
}
}  // namespace

// The device part of a grouped launch whose member table is already on the
// device: clear the claim counters, run the persistent contraction. Contains
// no allocation, copy or memset, so it can be captured in a graph and
// replayed.
hipError_t split_grouped_enqueue(void *ws, int count, const GroupedWork &work, hipStream_t st) {
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, st, static_cast<unsigned long long *>(ws));
    return launch_persistent(ws, count, work, st);
}

hipError_t launch_split_grouped(const moa_gemm_desc *const *members, int count, int variant, void *ws,
                                void *host_staging, const void *host_staging_dev, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const GroupedWork work = split_grouped_layout(members, count, ws, host_staging, variant);
    char *base = static_cast<char *>(ws);
    if (!host_staging_dev) {
        hipError_t e = hipMemcpyAsync(base + 256, host_staging, (size_t)work.table_used, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        return split_grouped_enqueue(ws, count, work, st);
    }
    const int64_t n16 = (work.table_used + 15) / 16;
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 64);
    hipLaunchKernelGGL(stage_table_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const uint4 *>(host_staging_dev), reinterpret_cast<uint4 *>(base + 256), n16,
                       reinterpret_cast<unsigned long long *>(base));
    return launch_persistent(ws, count, work, st);
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
