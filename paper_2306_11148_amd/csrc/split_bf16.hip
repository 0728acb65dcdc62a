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
// atomic counter until the list is exhausted. Every element of every member
// receives exactly the operation sequence of the single-product kernel (the
// per-element order depends only on the slab walk, not on the block shape),
// so grouped and single results are bitwise equal.
struct GroupMember {
    ring::Operands op;                  // the contraction's view (read by ring::tile in place)
    const float *A, *B;
    float *C;
    uint8_t *Ap, *Bp;                   // records of this member in the workspace
    int64_t m, n, p, S;
    int64_t first_tile;                 // first contraction work-list id of this member
    int64_t pack_first;                 // first conditioning work-list id of this member
    int32_t tiles_n, accumulate;
    int32_t row_items;                  // conditioning items: row_items chunk blocks of A,
    int32_t col_blocks_x;               // then col_blocks_x * ceil(S/4) 64 x 64 blocks of B
};


template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, 3) void split_grouped_kernel(
    const GroupMember *__restrict__ g, const int32_t *__restrict__ tile_owner, int64_t total_tiles,
    unsigned long long *__restrict__ counter) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[ring::Cfg<BM, BN, WM, WN, 1>::LDS];
    __shared__ int64_t s_tile;
    for (;;) {
        __syncthreads();                // nobody still reads lds or s_tile
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= total_tiles) break;
        const int k = __builtin_amdgcn_readfirstlane(tile_owner[tile]);
        const GroupMember &d = g[k];
        const int64_t local = tile - d.first_tile;
        const int64_t tm = local / d.tiles_n, tn = local - tm * d.tiles_n;
        ring::tile<BM, BN, WM, WN, 1, SplitMode>(d.op, __builtin_amdgcn_readfirstlane((int)tm) * (int64_t)BM,
                                                 __builtin_amdgcn_readfirstlane((int)tn) * (int64_t)BN, lds);
    }
}

// Grouped conditioning: one work list over every member, each member
// contributing row items (256 chunks of A each) followed by 64-column x 64-k
// blocks of B; workgroups stride through the list, so large and small members
// share the machine evenly. item_owner[item] names the member (a table built
// on the host: one load instead of a search through the member list).
constexpr int PACK_ROW_ITEM = 256;      // chunks per row item (one per thread)

__global__ __launch_bounds__(256) void grouped_pack_kernel(const GroupMember *__restrict__ g,
                                                           const int32_t *__restrict__ item_owner, int64_t total) {
    __shared__ __attribute__((aligned(16))) float tile[4 * SLAB][64 + 4];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int k = __builtin_amdgcn_readfirstlane(item_owner[item]);
        const GroupMember &d = g[k];
        const int64_t local = item - d.pack_first;
        if (local < d.row_items) {
            const int vec = (d.n % 8 == 0) && ((uintptr_t)d.A % 16 == 0);
            const int64_t q = local * PACK_ROW_ITEM + threadIdx.x;
            if (q < padded_rows(d.m) * d.S * 2) pack_rows_chunk(d.A, d.m, d.n, d.S, vec, d.Ap, q);
        } else {
            const int vec = (d.p % 4 == 0) && ((uintptr_t)d.B % 16 == 0);
            const int64_t b = local - d.row_items;
            pack_cols_block(d.B, d.n, d.p, d.S, d.Bp, b % d.col_blocks_x, b / d.col_blocks_x, tile, vec);
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
__global__ void zero_u64_kernel(unsigned long long *x) { *x = 0ull; }
constexpr int GB_M = 128, GB_N = 128, GW_M = 64, GW_N = 64;   // grouped block shape
int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
}  // namespace

namespace {
// Tiles and conditioning items of a member list (independent of the order).
GroupedWork grouped_counts(const moa_gemm_desc *const *members, int count) {
    GroupedWork w{0, 0};
    for (int k = 0; k < count; ++k) {
        const moa_gemm_desc &d = *members[k];
        const int64_t S = (d.n + SLAB - 1) / SLAB;
        w.tiles += ((d.m + GB_M - 1) / GB_M) * ((d.p + GB_N - 1) / GB_N);
        w.pack_items += (padded_rows(d.m) * S * 2 + PACK_ROW_ITEM - 1) / PACK_ROW_ITEM + ((d.p + 63) / 64) * ((S + 3) / 4);
    }
    return w;
}
// Member table, then tile -> member and item -> member tables (int32).
int64_t table_bytes(int count, const GroupedWork &w) {
    return align256((int64_t)count * (int64_t)sizeof(GroupMember)) + align256(4 * w.tiles) + align256(4 * w.pack_items);
}
}  // namespace

int64_t split_grouped_desc_bytes(const moa_gemm_desc *const *members, int count) {
    return table_bytes(count, grouped_counts(members, count));
}

int64_t split_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count) {
    int64_t b = 256 + split_grouped_desc_bytes(members, count);
    for (int k = 0; k < count; ++k)
        b += align256(split_bf16_workspace_bytes(members[k]->m, members[k]->n, members[k]->p));
    return b;
}

// Lays out the members (longest k walk first: the tail of the work list holds
// the cheapest tiles) in `host_staging` and the workspace; returns the tile
// count. The device member array is at ws + 256, the claim counter at ws.
GroupedWork split_grouped_layout(const moa_gemm_desc *const *members, int count, void *ws,
                                 void *host_staging) {
    std::vector<int> order(count);
    for (int k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return members[a]->n > members[b]->n;
    });
    const GroupedWork totals = grouped_counts(members, count);
    char *base = static_cast<char *>(ws);
    char *rec = base + 256 + table_bytes(count, totals);
    GroupMember *h = static_cast<GroupMember *>(host_staging);
    int32_t *tile_owner = reinterpret_cast<int32_t *>(static_cast<char *>(host_staging) +
                                                      align256((int64_t)count * (int64_t)sizeof(GroupMember)));
    int32_t *item_owner = tile_owner + align256(4 * totals.tiles) / 4;
    int64_t tiles = 0, items = 0;
    for (int q = 0; q < count; ++q) {
        const moa_gemm_desc &d = *members[order[q]];
        GroupMember g;
        g.A = static_cast<const float *>(d.A);
        g.B = static_cast<const float *>(d.B);
        g.C = static_cast<float *>(d.C);
        g.m = d.m; g.n = d.n; g.p = d.p;
        g.S = (d.n + SLAB - 1) / SLAB;
        g.Ap = reinterpret_cast<uint8_t *>(rec);
        g.Bp = g.Ap + ring::array_bytes(d.m, g.S);
        rec += align256(split_bf16_workspace_bytes(d.m, d.n, d.p));
        g.op = split_operands(g.Ap, g.Bp, g.C, d.m, d.p, g.S, d.accumulate);
        g.first_tile = tiles;
        g.tiles_n = (int32_t)((d.p + GB_N - 1) / GB_N);
        g.accumulate = d.accumulate;
        const int64_t mt = ((d.m + GB_M - 1) / GB_M) * g.tiles_n;
        for (int64_t t = 0; t < mt; ++t) tile_owner[tiles + t] = q;
        tiles += mt;
        g.pack_first = items;
        g.row_items = (int32_t)((padded_rows(d.m) * g.S * 2 + PACK_ROW_ITEM - 1) / PACK_ROW_ITEM);
        g.col_blocks_x = (int32_t)((d.p + 63) / 64);
        const int64_t mi = g.row_items + (int64_t)g.col_blocks_x * ((g.S + 3) / 4);
        for (int64_t t = 0; t < mi; ++t) item_owner[items + t] = q;
        items += mi;
        h[q] = g;
    }
    return {tiles, items};
}

// The device part of a grouped launch: reset the claim counter, condition
// every member, run the persistent contraction. Contains no allocation, copy
// or memset, so it can be captured in a graph and replayed.
hipError_t split_grouped_enqueue(void *ws, int count, const GroupedWork &work, hipStream_t st) {
    const int64_t tiles = work.tiles;
    char *base = static_cast<char *>(ws);
    unsigned long long *counter = reinterpret_cast<unsigned long long *>(base);
    const GroupMember *dev_members = reinterpret_cast<const GroupMember *>(base + 256);
    const int32_t *tile_owner = reinterpret_cast<const int32_t *>(
        base + 256 + align256((int64_t)count * (int64_t)sizeof(GroupMember)));
    const int32_t *item_owner = tile_owner + align256(4 * tiles) / 4;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, counter);
    if (work.pack_items > 0) {
        TraceScope ts(MOA_K_SPLIT_PACK, st);
        const int64_t g = std::min<int64_t>(work.pack_items, 8 * kNumCUs);
        hipLaunchKernelGGL(grouped_pack_kernel, dim3((unsigned)g), dim3(256), 0, st, dev_members, item_owner,
                           work.pack_items);
    }
    const int64_t grid = std::min<int64_t>(tiles, 3 * kNumCUs);   // three 48 KiB-LDS blocks per CU
    TraceScope ts(MOA_K_SPLIT_GROUPED, st);
    if (grid > 0)
        hipLaunchKernelGGL((split_grouped_kernel<GB_M, GB_N, GW_M, GW_N>), dim3((unsigned)grid),
                           dim3(ring::Cfg<GB_M, GB_N, GW_M, GW_N, 1>::THREADS), 0, st, dev_members, tile_owner,
                           tiles, counter);
    return hipGetLastError();
}

hipError_t launch_split_grouped(const moa_gemm_desc *const *members, int count, void *ws,
                                void *host_staging, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const GroupedWork work = split_grouped_layout(members, count, ws, host_staging);
    char *base = static_cast<char *>(ws);
    hipError_t e = hipMemcpyAsync(base + 256, host_staging, (size_t)split_grouped_desc_bytes(members, count),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return split_grouped_enqueue(ws, count, work, st);
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
