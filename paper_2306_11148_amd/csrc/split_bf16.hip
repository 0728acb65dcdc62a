// Split-BF16 matrix-core path: C = hi(A).hi(B) + hi(A).lo(B) + lo(A).hi(B)
// with FP32 accumulation, where x = hi + lo + O(2^-16 |x|), hi = RNE_bf16(x),
// lo = RNE_bf16(x - hi). This evaluates Eq. 3 (section "MoA Matrix
// Multiplication") to about FP32 accuracy on the BF16 matrix cores.
//
// Two stages.
//
// 1. Conditioning (HBM-bound): A and B are rewritten as "slab records". The k
//    extent is cut into slabs of 16 (the sigma loop broken into blocks,
//    section "Dimension Lifting to Machine Coordinates"); for every row i of
//    A and every column j of B, slab s becomes one contiguous 64-byte record
//        [hi of x[16s .. 16s+15] (16 bf16)][lo of the same (16 bf16)]
//    zero-padded past n. B is transposed on the way (column j of B becomes
//    record row j), so both operands are k-contiguous. Records are stored in
//    tiles of 16 rows x 1 slab: record (r, s) lives at byte
//        ((r / 16) * S + s) * 1024 + (r mod 16) * 64,
//    so the 16 records a wave moves into LDS in one load are one contiguous
//    KiB of whole cache lines. Row counts are padded to a multiple of 16 with
//    zero records.
//
// 2. Contraction (matrix-core bound), the blocked form of Fig. 2: each
//    workgroup owns a BM x BN block of C and walks the S slabs; per slab the
//    BM + BN records go straight from HBM into LDS (buffer_load ... lds, no
//    register staging) through a ring of NSTAGE buffers, so loads run
//    NSTAGE - 1 slabs ahead of the matrix cores. The block products of the slabs are
//    summed in registers (the "addition loop" over blocks). The fragments of
//    slab t+1 are read from LDS while the matrix-core steps of slab t issue.
//
// LDS holds one 64-byte row per record. gfx950's LDS serves a 16-byte read
// for 16 lanes per cycle out of a 256-byte bank window (64 banks), i.e. four
// consecutive rows at once. Chunk c of row r is stored at chunk position
// c ^ ((r / 4) mod 4): the 16 rows of one fragment-read cycle then occupy 16
// distinct 16-byte bank groups. The direct loads stay linear (lane L writes
// bytes 16L .. 16L+15 of its wave's 1 KiB window = 16 rows), so each lane
// fetches the logical chunk that belongs at its physical position.
#include <algorithm>
#include <vector>

#include "moa_internal.h"
#include "tile_common.h"

namespace moa {
namespace {

constexpr int SLAB = 16;                  // k per record
constexpr int REC = 2 * SLAB;             // bf16 per record (hi + lo)
constexpr int REC_BYTES = REC * 2;        // 64
constexpr int GROUP = 16;                 // rows per record tile (1 KiB per slab)

// bf16 offset of record (r, s) in a record array with S slabs per row
__device__ __forceinline__ int64_t rec_off(int64_t r, int64_t s, int64_t S) {
    return ((r / GROUP) * S + s) * (GROUP * REC) + (r % GROUP) * REC;
}
__host__ __device__ inline int64_t padded_rows(int64_t rows) { return (rows + GROUP - 1) / GROUP * GROUP; }
constexpr int NSTAGE = 3;                 // LDS ring depth (3 measured faster than 4 or 5)
// Two slabs per barrier (needs a 4-buffer ring): at even steps wait for the
// two slabs loaded at the previous barrier, refill the two buffers freed
// since, then run two slabs without a barrier.
constexpr bool PAIRED = false;

typedef __attribute__((address_space(3))) void lds_void_t;

// gfx9 s_waitcnt immediate that waits until at most n vector-memory
// operations of this wave are outstanding (expcnt and lgkmcnt not waited on).
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }

// Workgroup barrier without the release fence of __syncthreads(): that fence
// would also wait for the direct loads still in flight for later slabs. Each
// wave first waits (s_waitcnt) for its own loads of the slab it is about to
// read; LDS reads are complete before their values are used. The "memory"
// clobber keeps the compiler from moving LDS accesses across the barrier.
__device__ __forceinline__ void ring_barrier() { asm volatile("s_barrier" ::: "memory"); }

// ---------------------------------------------------------------- stage 1 --

// Rows of X (rows x K, row-major) -> records: chunk q = 8 k values of one
// record (2 chunks per record).
__device__ __forceinline__ void pack_rows_chunk(const float *__restrict__ X, int64_t rows, int64_t K,
                                                int64_t S, int vec, uint16_t *__restrict__ P,
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
    uint16_t *rec = P + rec_off(r, s, S);
    *reinterpret_cast<uint4 *>(rec + c * 8) = hi;
    *reinterpret_cast<uint4 *>(rec + SLAB + c * 8) = lo;
}

__global__ __launch_bounds__(256) void pack_rows_kernel(const float *__restrict__ X, int64_t rows,
                                                        int64_t K, int64_t S, int vec,
                                                        uint16_t *__restrict__ P) {
    const int64_t chunks = padded_rows(rows) * S * 2;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256)
        pack_rows_chunk(X, rows, K, S, vec, P, q);
}

// Columns of X (K x cols, row-major) -> records (transposed). Block (bx, by)
// covers columns 64 bx .. 64 bx + 63 and slabs 4 by .. 4 by + 3; it goes
// through LDS so that reads of X rows are contiguous and every wave store
// writes one whole KiB record tile. Columns past `cols` get zero records.
// All 256 threads must call it together.
// Columns of X (K x cols, row-major) -> records (transposed), 64 columns x
// 64 k (4 slabs) per block through LDS: reads of X rows are contiguous
// float4s and each thread writes one whole 64-byte record. Columns past
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
__device__ __forceinline__ void pack_cols_emit(const ColBlockRegs &r, int64_t cols, int64_t S,
                                               uint16_t *__restrict__ P, int64_t bx, int64_t by,
                                               float (*tile)[64 + 4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        *reinterpret_cast<float4 *>(&tile[(t >> 4) + 16 * i][(t & 15) * 4]) = r.v[i];
    __syncthreads();
    const int jj = t & 63, part = t >> 6;
    const int64_t j = bx * 64 + jj, s = by * 4 + part;
    if (j < padded_rows(cols) && s < S) {
        uint4 h[2], l[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int kb = part * SLAB + c * 8;
            split_pair(tile[kb + 0][jj], tile[kb + 1][jj], &h[c].x, &l[c].x);
            split_pair(tile[kb + 2][jj], tile[kb + 3][jj], &h[c].y, &l[c].y);
            split_pair(tile[kb + 4][jj], tile[kb + 5][jj], &h[c].z, &l[c].z);
            split_pair(tile[kb + 6][jj], tile[kb + 7][jj], &h[c].w, &l[c].w);
        }
        uint4 *rec = reinterpret_cast<uint4 *>(P + rec_off(j, s, S));
        rec[0] = h[0];
        rec[1] = h[1];
        rec[2] = l[0];
        rec[3] = l[1];
    }
    __syncthreads();                             // tile free for the next block
}

__device__ __forceinline__ void pack_cols_block(const float *__restrict__ X, int64_t K, int64_t cols,
                                                int64_t S, uint16_t *__restrict__ P, int64_t bx,
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
                                                        uint16_t *__restrict__ P) {
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

// Geometry of one block configuration.
template <int BM, int BN, int WM, int WN> struct TileCfg {
    static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN, NW = WAVES_M * WAVES_N;
    static constexpr int THREADS = NW * 64;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int ROWS = BM + BN;                  // records per slab
    static constexpr int STAGE = ROWS * REC_BYTES;        // bytes per LDS buffer
    static constexpr int LDS = NSTAGE * STAGE;
    static constexpr int LPW = ROWS / 16 / NW;            // 1 KiB direct loads per wave per slab
    static_assert(ROWS % (16 * NW) == 0 && BM % 16 == 0, "whole loads per wave");
};

// One BM x BN block of C at (i0, j0): the whole k walk and the epilogue.
// `lds` is the workgroup's ring of NSTAGE buffers. On entry no wave may still
// be reading `lds` (the caller's barrier); on exit every wave has finished.
template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void split_tile(const uint16_t *__restrict__ Ap,
                                           const uint16_t *__restrict__ Bp, float *__restrict__ C,
                                           int64_t m, int64_t p, int64_t S, int accumulate,
                                           int64_t i0, int64_t j0, uint8_t *lds) {
    using G = TileCfg<BM, BN, WM, WN>;
    constexpr int WAVES_N = G::WAVES_N, FM = G::FM, FN = G::FN;
    constexpr int STAGE = G::STAGE, LPW = G::LPW;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;

    // Direct loads through two buffer resources based at this tile's first
    // record row of A and of B. Load Q = wave*LPW + q fills LDS rows
    // 16Q .. 16Q+15: lane L lands at row 16Q + L/4, physical chunk L%4, and
    // fetches logical chunk (L%4) ^ ((row/4) mod 4) = (L%4) ^ (L/16). The row
    // block and the slab go in the uniform soffset. Records past m (or p) lie
    // beyond the resource's range and load as zeros (their outputs are not
    // stored).
    const int64_t tile_row = S * GROUP * REC_BYTES;   // bytes per row tile (16 rows, all slabs)
    const int64_t tiles_a = min((int64_t)BM, padded_rows(m) - i0) / GROUP;
    const int64_t tiles_b = min((int64_t)BN, padded_rows(p) - j0) / GROUP;
    const __amdgpu_buffer_rsrc_t rsrc_a = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(reinterpret_cast<const uint8_t *>(Ap) + (i0 / GROUP) * tile_row), (short)0,
        (int)(tiles_a * tile_row), 0x00020000);
    const __amdgpu_buffer_rsrc_t rsrc_b = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(reinterpret_cast<const uint8_t *>(Bp) + (j0 / GROUP) * tile_row), (short)0,
        (int)(tiles_b * tile_row), 0x00020000);
    const int voff = (lane >> 2) * REC_BYTES + (((lane & 3) ^ (lane >> 4)) << 4);
    // Each wave's LPW loads cover 16*LPW consecutive rows that are either
    // all rows of A or all rows of B, so every load names one resource.
    static_assert(BM % (16 * LPW) == 0, "a wave loads A rows or B rows, not both");
    const bool loads_a = wave * LPW * 16 < BM;
    const int row_base = loads_a ? wave * LPW * 16 : wave * LPW * 16 - BM;
    auto issue = [&](int64_t s) {
        uint8_t *buf = lds + (int)(s % NSTAGE) * STAGE + wave * LPW * 16 * REC_BYTES;
        if (loads_a) {
#pragma unroll
            for (int q = 0; q < LPW; ++q)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsrc_a, (lds_void_t *)(buf + q * 16 * REC_BYTES), 16, voff,
                    (int)((row_base / GROUP + q) * tile_row + s * GROUP * REC_BYTES), 0, 0);
        } else {
#pragma unroll
            for (int q = 0; q < LPW; ++q)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsrc_b, (lds_void_t *)(buf + q * 16 * REC_BYTES), 16, voff,
                    (int)((row_base / GROUP + q) * tile_row + s * GROUP * REC_BYTES), 0, 0);
        }
    };

    // Fragment of 32 records (rows) x 8 k: lane l reads logical chunk c of
    // row base + l%32; hi is chunk l/32, lo is chunk 2 + l/32.
    const int frow = lane & 31, fhalf = lane >> 5;
    auto frag = [&](const uint8_t *buf, int row, int chunk) {
        return *reinterpret_cast<const bf16x8_t *>(buf + row * REC_BYTES +
                                                   ((chunk ^ ((row >> 2) & 3)) << 4));
    };
    struct Frags { bf16x8_t ah[FM], al[FM], bh[FN], bl[FN]; };
    auto read_frags = [&](int64_t s, Frags &f) {
        const uint8_t *buf = lds + (int)(s % NSTAGE) * STAGE;
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            const int row = wm * WM + a * 32 + frow;
            f.ah[a] = frag(buf, row, fhalf);
            f.al[a] = frag(buf, row, 2 + fhalf);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int row = BM + wn * WN + b * 32 + frow;
            f.bh[b] = frag(buf, row, fhalf);
            f.bl[b] = frag(buf, row, 2 + fhalf);
        }
    };

    f32x16_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16_t{};

    // term-major order: consecutive matrix-core steps are independent
    auto mma = [&](const Frags &f) {
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
    };

    // One step: make slab t+1 visible, refill the buffer slab t-1 used with
    // slab t+3, read slab t+1's fragments, then issue slab t's products.
    // Wait until at most `stages` slabs of this wave's loads are still in
    // flight (the immediate of s_waitcnt must be a constant).
    auto wait_loads = [&](int64_t stages) {
        switch (stages <= 0 ? 0 : stages >= 3 ? 3 : (int)stages) {
        case 0: __builtin_amdgcn_s_waitcnt(waitcnt_vm(0)); break;
        case 1: __builtin_amdgcn_s_waitcnt(waitcnt_vm(LPW)); break;
        case 2: __builtin_amdgcn_s_waitcnt(waitcnt_vm(2 * LPW)); break;
        default: __builtin_amdgcn_s_waitcnt(waitcnt_vm(3 * LPW)); break;
        }
    };
    static_assert(NSTAGE >= 3 && NSTAGE <= 5, "wait_loads covers up to 3 slabs in flight");

    // One step: make slab t+1 visible (its loads landed in every wave), refill
    // the buffer slab t-1 used with slab t+NSTAGE-1, read slab t+1's
    // fragments, then issue slab t's products.
    auto step = [&](int64_t t, const Frags &cur, Frags &next) {
        if (t + 1 < S) {
            // issued so far: slabs up to t + NSTAGE - 2; t + 1 must have landed
            wait_loads(min((int64_t)NSTAGE - 3, S - t - 2));
            ring_barrier();
            if (t + NSTAGE - 1 < S) issue(t + NSTAGE - 1);
            read_frags(t + 1, next);
        }
        mma(cur);
    };

    if (S > 0 && !PAIRED) {
        for (int q = 0; q < NSTAGE - 1; ++q)
            if (q < S) issue(q);
        wait_loads(min((int64_t)NSTAGE - 2, S - 1));   // slab 0 has landed
        ring_barrier();
        Frags f0, f1;
        read_frags(0, f0);
        int64_t t = 0;
        for (; t + 1 < S; t += 2) {
            step(t, f0, f1);
            step(t + 1, f1, f0);
        }
        if (t < S) step(t, f0, f1);
    } else if (S > 0) {
        static_assert(!PAIRED || NSTAGE == 4, "paired barriers use a 4-buffer ring");
        for (int q = 0; q < 3; ++q)
            if (q < S) issue(q);
        wait_loads(min((int64_t)2, S - 1));            // slab 0 has landed
        ring_barrier();
        Frags f0, f1;
        read_frags(0, f0);
        for (int64_t t = 0; t < S; t += 2) {
            if (t + 1 < S) {
                wait_loads(0);                         // slabs t+1, t+2 have landed
                ring_barrier();
                if (t + 3 < S) issue(t + 3);           // into the buffers of slabs t-1 and t,
                if (t + 4 < S) issue(t + 4);           // whose fragments are in registers
                read_frags(t + 1, f1);
            }
            mma(f0);
            if (t + 1 < S) {
                if (t + 2 < S) read_frags(t + 2, f0);
                mma(f1);
            }
        }
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

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void split_bf16_kernel(
    const uint16_t *__restrict__ Ap, const uint16_t *__restrict__ Bp, float *__restrict__ C,
    int64_t m, int64_t p, int64_t S, int accumulate, int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TileCfg<BM, BN, WM, WN>::LDS];
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, &tm, &tn);
    // the integer divisions above run on the vector ALU; pin the (uniform)
    // results to scalar registers so everything derived from them stays scalar
    tm = __builtin_amdgcn_readfirstlane(tm);
    tn = __builtin_amdgcn_readfirstlane(tn);
    split_tile<BM, BN, WM, WN>(Ap, Bp, C, m, p, S, accumulate, (int64_t)tm * BM, (int64_t)tn * BN, lds);
}

// ------------------------------------------------------- grouped (persistent)
// Independent products share one launch. Members are listed longest k walk
// first; their tiles form one work list (member g owns tile ids
// [first[g], first[g+1])), and persistent workgroups claim tile ids from an
// atomic counter until the list is exhausted. Every element of every member
// receives exactly the operation sequence of the single-product kernel (the
// per-element order depends only on the slab walk, not on the block shape),
// so grouped and single results are bitwise equal.
struct GroupMember {
    const float *A, *B;
    float *C;
    uint16_t *Ap, *Bp;                  // records of this member in the workspace
    int64_t m, n, p, S;
    int64_t first_tile;                 // first work-list id of this member
    int32_t tiles_n, accumulate;
};

__device__ __forceinline__ int find_member(const GroupMember *__restrict__ g, int count, int64_t tile) {
    int lo = 0, hi = count - 1;         // last member with first_tile <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g[mid].first_tile <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void split_grouped_kernel(
    const GroupMember *__restrict__ g, int count, int64_t total_tiles,
    unsigned long long *__restrict__ counter) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TileCfg<BM, BN, WM, WN>::LDS];
    __shared__ int64_t s_tile;
    for (;;) {
        __syncthreads();                // nobody still reads lds or s_tile
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= total_tiles) break;
        const int k = __builtin_amdgcn_readfirstlane(find_member(g, count, tile));
        const GroupMember &d = g[k];
        const int64_t local = tile - d.first_tile;
        const int64_t tm = local / d.tiles_n, tn = local - tm * d.tiles_n;
        split_tile<BM, BN, WM, WN>(d.Ap, d.Bp, d.C, d.m, d.p, d.S, d.accumulate,
                                   __builtin_amdgcn_readfirstlane((int)tm) * (int64_t)BM,
                                   __builtin_amdgcn_readfirstlane((int)tn) * (int64_t)BN, lds);
    }
}

// Grouped conditioning: each workgroup walks a share of every member's
// chunks (rows of A) and 64 x 64 blocks (columns of B).
__global__ __launch_bounds__(256) void grouped_pack_rows_kernel(const GroupMember *__restrict__ g,
                                                                int count) {
    for (int k = blockIdx.y; k < count; k += gridDim.y) {
        const GroupMember d = g[k];
        const int vec = (d.n % 8 == 0) && ((uintptr_t)d.A % 16 == 0);
        const int64_t chunks = padded_rows(d.m) * d.S * 2;
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * 256)
            pack_rows_chunk(d.A, d.m, d.n, d.S, vec, d.Ap, q);
    }
}

__global__ __launch_bounds__(256) void grouped_pack_cols_kernel(const GroupMember *__restrict__ g,
                                                                int count) {
    __shared__ __attribute__((aligned(16))) float tile[4 * SLAB][64 + 4];
    for (int k = blockIdx.y; k < count; k += gridDim.y) {
        const GroupMember d = g[k];
        const int vec = (d.p % 4 == 0) && ((uintptr_t)d.B % 16 == 0);
        const int64_t bx = (d.p + 63) / 64, by = (d.S + 3) / 4;
        for (int64_t b = blockIdx.x; b < bx * by; b += gridDim.x) {
            __syncthreads();
            pack_cols_block(d.B, d.n, d.p, d.S, d.Bp, b % bx, b / bx, tile, vec);
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
constexpr SplitShape kSplit[] = {{128, 128, 64, 64}, {256, 256, 128, 64}};

template <int BM, int BN, int WM, int WN>
hipError_t launch_shape(const moa_gemm_desc &d, const uint16_t *Ap, const uint16_t *Bp, int64_t S,
                        hipStream_t st) {
    float *C = static_cast<float *>(d.C);
    const int tiles_m = (int)((d.m + BM - 1) / BM);
    const int tiles_n = (int)((d.p + BN - 1) / BN);
    constexpr int threads = (BM / WM) * (BN / WN) * 64;
    hipLaunchKernelGGL((split_bf16_kernel<BM, BN, WM, WN>), dim3(tiles_m * tiles_n), dim3(threads), 0,
                       st, Ap, Bp, C, d.m, d.p, S, d.accumulate, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace

int split_bf16_variant_count() { return (int)(sizeof(kSplit) / sizeof(kSplit[0])); }

int64_t split_bf16_workspace_bytes(int64_t m, int64_t n, int64_t p) {
    const int64_t S = (n + SLAB - 1) / SLAB;
    return (padded_rows(m) + padded_rows(p)) * S * REC_BYTES;
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
    p->lds_bytes = NSTAGE * (s.bm + s.bn) * REC_BYTES;
}

hipError_t launch_split_pack(const moa_gemm_desc &d, void *ws, hipStream_t st) {
    const int64_t S = (d.n + SLAB - 1) / SLAB;
    uint16_t *Ap = static_cast<uint16_t *>(ws);
    uint16_t *Bp = Ap + padded_rows(d.m) * S * REC;
    const float *A = static_cast<const float *>(d.A);
    const float *B = static_cast<const float *>(d.B);
    if (S == 0) return hipSuccess;
    const int vec = (d.n % 8 == 0) && ((uintptr_t)A % 16 == 0);
    const int64_t chunks = padded_rows(d.m) * S * 2;
    int64_t blocks = (chunks + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, d.m, d.n, S, vec, Ap);
    const int vec_b = (d.p % 4 == 0) && ((uintptr_t)B % 16 == 0);
    const int64_t by = ((S + 3) / 4 + COL_BLOCKS - 1) / COL_BLOCKS;
    hipLaunchKernelGGL(pack_cols_kernel, dim3((unsigned)((d.p + 63) / 64), (unsigned)(by < 65535 ? by : 65535)),
                       dim3(256), 0, st, B, d.n, d.p, S, vec_b, Bp);
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
    const uint16_t *Ap = static_cast<const uint16_t *>(ws);
    const uint16_t *Bp = Ap + padded_rows(d.m) * S * REC;
    switch (plan.variant) {
    case 0: return launch_shape<128, 128, 64, 64>(d, Ap, Bp, S, st);
    default: return launch_shape<256, 256, 128, 64>(d, Ap, Bp, S, st);
    }
}

namespace {
__global__ void zero_u64_kernel(unsigned long long *x) { *x = 0ull; }
constexpr int GB_M = 128, GB_N = 128, GW_M = 64, GW_N = 64;   // grouped block shape
int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
}  // namespace

int64_t split_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count) {
    int64_t b = 256 + align256((int64_t)count * (int64_t)sizeof(GroupMember));
    for (int k = 0; k < count; ++k)
        b += align256(split_bf16_workspace_bytes(members[k]->m, members[k]->n, members[k]->p));
    return b;
}

int64_t split_grouped_desc_bytes(int count) { return (int64_t)count * (int64_t)sizeof(GroupMember); }

// Lays out the members (longest k walk first: the tail of the work list holds
// the cheapest tiles) in `host_staging` and the workspace; returns the tile
// count. The device member array is at ws + 256, the claim counter at ws.
int64_t split_grouped_layout(const moa_gemm_desc *const *members, int count, void *ws,
                             void *host_staging) {
    std::vector<int> order(count);
    for (int k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return members[a]->n > members[b]->n;
    });
    char *base = static_cast<char *>(ws);
    char *rec = base + 256 + align256((int64_t)count * (int64_t)sizeof(GroupMember));
    GroupMember *h = static_cast<GroupMember *>(host_staging);
    int64_t tiles = 0;
    for (int q = 0; q < count; ++q) {
        const moa_gemm_desc &d = *members[order[q]];
        GroupMember g;
        g.A = static_cast<const float *>(d.A);
        g.B = static_cast<const float *>(d.B);
        g.C = static_cast<float *>(d.C);
        g.m = d.m; g.n = d.n; g.p = d.p;
        g.S = (d.n + SLAB - 1) / SLAB;
        g.Ap = reinterpret_cast<uint16_t *>(rec);
        g.Bp = g.Ap + padded_rows(d.m) * g.S * REC;
        rec += align256(split_bf16_workspace_bytes(d.m, d.n, d.p));
        g.first_tile = tiles;
        g.tiles_n = (int32_t)((d.p + GB_N - 1) / GB_N);
        g.accumulate = d.accumulate;
        tiles += ((d.m + GB_M - 1) / GB_M) * g.tiles_n;
        h[q] = g;
    }
    return tiles;
}

// The device part of a grouped launch: reset the claim counter, condition
// every member, run the persistent contraction. Contains no allocation, copy
// or memset, so it can be captured in a graph and replayed.
hipError_t split_grouped_enqueue(void *ws, int count, int64_t tiles, hipStream_t st) {
    char *base = static_cast<char *>(ws);
    unsigned long long *counter = reinterpret_cast<unsigned long long *>(base);
    const GroupMember *dev_members = reinterpret_cast<const GroupMember *>(base + 256);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, counter);
    const unsigned gy = (unsigned)std::min(count, 65535);
    {
        TraceScope ts(MOA_K_SPLIT_PACK, st);
        hipLaunchKernelGGL(grouped_pack_rows_kernel, dim3(32, gy), dim3(256), 0, st, dev_members, count);
        hipLaunchKernelGGL(grouped_pack_cols_kernel, dim3(16, gy), dim3(256), 0, st, dev_members, count);
    }
    const int64_t grid = std::min<int64_t>(tiles, 2 * kNumCUs);   // two 64 KiB-LDS blocks per CU
    TraceScope ts(MOA_K_SPLIT_GROUPED, st);
    if (grid > 0)
        hipLaunchKernelGGL((split_grouped_kernel<GB_M, GB_N, GW_M, GW_N>), dim3((unsigned)grid),
                           dim3(TileCfg<GB_M, GB_N, GW_M, GW_N>::THREADS), 0, st, dev_members, count,
                           tiles, counter);
    return hipGetLastError();
}

hipError_t launch_split_grouped(const moa_gemm_desc *const *members, int count, void *ws,
                                void *host_staging, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t tiles = split_grouped_layout(members, count, ws, host_staging);
    char *base = static_cast<char *>(ws);
    hipError_t e = hipMemcpyAsync(base + 256, host_staging, (size_t)count * sizeof(GroupMember),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return split_grouped_enqueue(ws, count, tiles, st);
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
