// Blocked matrix-core contraction over conditioned "record tiles", shared by
// the split-BF16 and scaled-FP8 paths.
//
// Conditioned operands: for every row i of A and every column j of B, the k
// extent is cut into slabs (the sigma loop broken into blocks, section
// "Dimension Lifting to Machine Coordinates" of the paper) and slab s of that
// row becomes one 64-byte record. Records are stored in tiles of 16 rows x 1
// slab: record (r, s) lives at byte ((r / 16) * S + s) * 1024 + (r mod 16) * 64,
// so 16 records are one contiguous KiB of whole cache lines. Row counts are
// padded to a multiple of 16 with zero records. A path may keep NREC record
// arrays per operand (e.g. a high and a low term).
//
// Contraction (Fig. 2 blocking): a workgroup owns a BM x BN block of C and
// walks the S slabs; per slab the NREC*(BM+BN) records go straight from HBM
// into LDS (buffer_load ... lds, no register staging) through a ring of
// NSTAGE buffers, and the slab's block products are summed in registers (the
// "addition loop" over blocks). The fragments of slab t+1 are read from LDS
// while the matrix-core steps of slab t issue.
//
// LDS holds one 64-byte row per record. gfx950's LDS serves a 16-byte read for
// 16 lanes per cycle out of a 256-byte window (64 banks), i.e. four
// consecutive rows at once: chunk c of row r is stored at chunk position
// c ^ ((r / 4) mod 4), so the 16 rows of a read cycle hit 16 distinct bank
// groups. The direct loads stay linear (lane L writes bytes 16L .. 16L+15 of
// its wave's KiB window = 16 rows), so each lane fetches the logical chunk
// that belongs at its physical position.
#pragma once

#include <algorithm>
#include <type_traits>

#include "moa_internal.h"
#include "tile_common.h"

namespace moa {
namespace ring {

constexpr int REC_BYTES = 64;             // bytes per record
constexpr int GROUP = 16;                 // rows per record tile
constexpr int NSTAGE = 3;                 // default LDS ring depth (slabs in LDS at once)

__host__ __device__ inline int64_t padded_rows(int64_t rows) { return (rows + GROUP - 1) / GROUP * GROUP; }

// byte offset of record (r, s) in a record array with S slabs per row
__host__ __device__ inline int64_t rec_byte(int64_t r, int64_t s, int64_t S) {
    return ((r / GROUP) * S + s) * (GROUP * REC_BYTES) + (r % GROUP) * REC_BYTES;
}

// bytes of one record array for `rows` rows and S slabs
__host__ __device__ inline int64_t array_bytes(int64_t rows, int64_t S) { return padded_rows(rows) * S * REC_BYTES; }

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) float global_f32;
typedef __attribute__((address_space(1))) const int32_t global_i32;

// gfx9 s_waitcnt immediate: at most n vector-memory operations of this wave
// outstanding (expcnt and lgkmcnt not waited on).
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }

// Workgroup barrier without the release fence of __syncthreads(): that fence
// would also wait for the direct loads still in flight for later slabs. Each
// wave first waits (s_waitcnt) for its own loads of the slab it is about to
// read; LDS reads are complete before their values are used. The "memory"
// clobber keeps the compiler from moving LDS accesses across the barrier.
__device__ __forceinline__ void ring_barrier() { asm volatile("s_barrier" ::: "memory"); }

template <int BM, int BN, int WM, int WN, int NREC, int NST = NSTAGE> struct Cfg {
    static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN, NW = WAVES_M * WAVES_N;
    static constexpr int THREADS = NW * 64;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int ROWS = NREC * (BM + BN);         // records per slab
    static constexpr int STAGE = ROWS * REC_BYTES;        // bytes per LDS buffer
    static constexpr int LDS = NST * STAGE;
    static constexpr int LPW = ROWS / 16 / NW;            // KiB direct loads per wave per slab
    static_assert(ROWS % (16 * NW) == 0, "whole loads per wave");
    // a wave's rows lie in one array, or span two (then fewer rows than either array)
    static constexpr bool ONE_ARRAY = BM % (16 * LPW) == 0 && BN % (16 * LPW) == 0;
    static_assert(ONE_ARRAY || (16 * LPW <= BM && 16 * LPW <= BN), "a wave's rows span at most two arrays");
};

// Vector offset of a load that must touch no memory: beyond any resource
// range (records per resource stay below 2^31 bytes).
constexpr int kDeadVoffset = (int)0x80000000u;

// Where LDS row `row` of a slab comes from (rows: [A array 0 (BM)] ..
// [A array NREC-1] [B array 0 (BN)] ..): operand A or B, record array, the
// row's index inside the block's part of that array, the block's first row
// tile of the array and how many 16-row tiles of it exist from there (the
// block may overhang the padded end). Shared by the kernels and the host
// check of their loads (check_loads).
struct RowWindow {
    bool a;
    int arr, row_in, tiles;
    int64_t first_tile;
};
__host__ __device__ inline RowWindow row_window(int BM, int BN, int NREC, int row, int64_t i0, int64_t j0, int64_t m,
                                                int64_t p) {
    RowWindow w;
    w.a = row < NREC * BM;
    w.arr = NREC == 1 ? 0 : w.a ? row / BM : (row - NREC * BM) / BN;
    w.row_in = w.a ? row - w.arr * BM : row - NREC * BM - w.arr * BN;
    const int64_t org = w.a ? i0 : j0;
    const int64_t left = padded_rows(w.a ? m : p) - org;
    const int64_t span = w.a ? BM : BN;
    w.first_tile = org / GROUP;
    w.tiles = (int)((left < span ? left : span) / GROUP);
    return w;
}
// The first of a wave's LPW loads whose rows lie in the next array (LPW when
// they all lie in one).
__host__ __device__ inline int q_split_of(int BM, int BN, int NREC, int LPW, bool one_array, int row_first) {
    if (one_array) return LPW;
    const int end0 = row_first < NREC * BM ? (row_first / BM + 1) * BM
                                           : NREC * BM + ((row_first - NREC * BM) / BN + 1) * BN;
    const int q = (end0 - row_first) / 16;
    return q < LPW ? q : LPW;
}

// The conditioned operands of one product.
struct Operands {
    const uint8_t *a0, *a1;               // record arrays of A (a1 only when NREC == 2)
    const uint8_t *b0, *b1;               // record arrays of B
    float *C;
    const int32_t *row_exp;               // scaled modes: C[i][j] = 2^-(row_exp[i] + col_exp[j]) acc
    const int32_t *col_exp;
    int64_t m, p, S;
    int accumulate;
};

// Fragment read of 16 bytes from LDS: logical chunk `chunk` of row `row`.
template <class V>
__device__ __forceinline__ V lds_chunk(const uint8_t *buf, int row, int chunk) {
    static_assert(sizeof(V) == 16, "one 16-byte chunk");
    return *reinterpret_cast<const V *>(buf + row * REC_BYTES + ((chunk ^ ((row >> 2) & 3)) << 4));
}

// One BM x BN block of C at (i0, j0). Mode supplies
//   template <int FM, int FN> struct Frags         fragments of one slab
//   template <int BM, int BN, int FM, int FN>
//   static void read(buf, a_row, b_row, half, Frags &)   LDS -> registers
//   template <int FM, int FN> static void mma(const Frags &, acc)
//   static constexpr bool SCALED                   apply row/col exponents
// and the LDS rows of a slab are [A array 0 (BM)] .. [A array NREC-1]
// [B array 0 (BN)] .. [B array NREC-1].
// `lds` is the workgroup's ring; on entry no wave may still be reading it, on
// exit every wave has finished.
// The k walk covers slabs s_begin .. s_end-1 (all slabs by default). With
// `partial` set, the epilogue stores the raw block sum there (row-major m x p,
// no descale, no accumulate): one chunk of a split-k product.
template <int BM, int BN, int WM, int WN, int NREC, class Mode, int NSTAGE = ring::NSTAGE>
__device__ __forceinline__ void tile(const Operands &op, int64_t i0, int64_t j0, uint8_t *lds, int s_begin = 0,
                                     int s_end = -1, float *partial = nullptr) {
    using G = Cfg<BM, BN, WM, WN, NREC, NSTAGE>;
    constexpr int WAVES_N = G::WAVES_N, FM = G::FM, FN = G::FN;
    constexpr int STAGE = G::STAGE, LPW = G::LPW;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int S = (int)op.S;                 // the planner keeps S below 2^17
    const int s0 = s_begin;
    const int L = (s_end < 0 ? S : s_end) - s_begin;   // slabs this block walks

    // LDS rows of a slab: [A array 0 (BM)] .. [A array NREC-1] [B array 0 (BN)] ..
    // Wave w loads rows 16*LPW*w .. +16*LPW-1: inside one array, or (when the
    // block's arrays are not multiples of a wave's share) across the end of
    // one array into the next, from loads q_split onwards.
    static_assert(NREC == 1 || NREC == 2, "one or two record arrays per operand");
    const int64_t tile_row = S * GROUP * REC_BYTES;       // bytes per row tile (16 rows, all slabs)
    const int row_first = wave * LPW * 16;
    // A buffer resource over the block's row tiles of the array holding a
    // window's rows. (with two arrays the select of the base becomes a
    // variable index into `op`: keep `op` in kernel-argument or global memory,
    // never in a local variable, or it is placed in scratch memory)
    auto resource = [&](const RowWindow &w) {
        const uint8_t *base = w.a ? (NREC == 1 || w.arr == 0 ? op.a0 : op.a1) : (NREC == 1 || w.arr == 0 ? op.b0 : op.b1);
        return __builtin_amdgcn_make_buffer_rsrc((void *)(base + w.first_tile * tile_row), (short)0,
                                                 (int)(w.tiles * tile_row), 0x00020000);
    };
    const RowWindow w0 = row_window(BM, BN, NREC, row_first, i0, j0, op.m, op.p);
    const __amdgpu_buffer_rsrc_t rsrc0 = resource(w0);
    const int q_split = q_split_of(BM, BN, NREC, LPW, G::ONE_ARRAY, row_first);
    RowWindow w1 = w0;
    __amdgpu_buffer_rsrc_t rsrc1 = rsrc0;
    if constexpr (!G::ONE_ARRAY) {
        if (q_split < LPW) {
            w1 = row_window(BM, BN, NREC, row_first + 16 * q_split, i0, j0, op.m, op.p);
            rsrc1 = resource(w1);
        }
    }
    // lane L lands at row 16Q + L/4, physical chunk L%4, and fetches logical
    // chunk (L%4) ^ ((row/4) mod 4) = (L%4) ^ (L/16). Rows of the last
    // partial tile past m (or p) are zero records written by the conditioning.
    // A load whose whole 16-row tile lies past the padded end of its array
    // (the block overhangs the operand) gets the vector offset 2^31, beyond
    // the resource's range (below 2^31 bytes), so it touches no memory whether
    // or not the range check counts the scalar offset (below 2^31 too, so the
    // sum does not wrap); its LDS rows feed only outputs past m or p, which
    // are never stored.
    const int voff = (lane >> 2) * REC_BYTES + (((lane & 3) ^ (lane >> 4)) << 4);
    auto issue = [&](int s) {            // s counts from s_begin
        uint8_t *buf = lds + (s % NSTAGE) * STAGE + row_first * REC_BYTES;
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const bool first = G::ONE_ARRAY || q < q_split;
            const int tile_in = first ? w0.row_in / GROUP + q : w1.row_in / GROUP + (q - q_split);
            const bool live = tile_in < (first ? w0.tiles : w1.tiles);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                first ? rsrc0 : rsrc1, (lds_void_t *)(buf + q * 16 * REC_BYTES), 16,
                live ? voff : kDeadVoffset, (int)(tile_in * tile_row) + (s0 + s) * GROUP * REC_BYTES, 0, 0);
        }
    };

    const int frow = lane & 31, fhalf = lane >> 5;
    typename Mode::template Frags<FM, FN> f0, f1;
    auto read = [&](int s, typename Mode::template Frags<FM, FN> &f) {
        const uint8_t *buf = lds + (s % NSTAGE) * STAGE;
        Mode::template read<BM, BN, FM, FN>(buf, wm * WM + frow, NREC * BM + wn * WN + frow, fhalf, f);
    };

    f32x16_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16_t{};

    // Wait until at most `stages` slabs of this wave's loads are in flight.
    auto wait_loads = [&](int stages) {
        switch (stages <= 0 ? 0 : stages >= 3 ? 3 : stages) {
        case 0: __builtin_amdgcn_s_waitcnt(waitcnt_vm(0)); break;
        case 1: __builtin_amdgcn_s_waitcnt(waitcnt_vm(LPW)); break;
        case 2: __builtin_amdgcn_s_waitcnt(waitcnt_vm(2 * LPW)); break;
        default: __builtin_amdgcn_s_waitcnt(waitcnt_vm(3 * LPW)); break;
        }
    };
    static_assert(NSTAGE >= 3 && NSTAGE <= 5, "wait_loads covers up to 3 slabs in flight");
    static_assert(3 * LPW <= 63, "vmcnt counts up to 63 operations");

    // One step (slab t + 1 exists): make slab t+1 visible (its loads landed
    // in every wave), refill the buffer slab t-1 used with slab t+NSTAGE-1,
    // read slab t+1's fragments, then issue slab t's products. The read is
    // unconditional so that the two fragment sets keep fixed registers.
    auto step = [&](int t, const typename Mode::template Frags<FM, FN> &cur,
                    typename Mode::template Frags<FM, FN> &next) {
        // issued so far: slabs up to t + NSTAGE - 2; t + 1 must have landed
        wait_loads(min(NSTAGE - 3, L - t - 2));
        ring_barrier();
        if (t + NSTAGE - 1 < L) issue(t + NSTAGE - 1);
        read(t + 1, next);
        Mode::template mma<FM, FN>(cur, acc);
    };

    if (L > 0) {
        for (int q = 0; q < NSTAGE - 1; ++q)
            if (q < L) issue(q);
        wait_loads(min(NSTAGE - 2, L - 1));            // slab 0 has landed
        ring_barrier();
        read(0, f0);
        int t = 0;
        for (; t + 2 < L; t += 2) {
            step(t, f0, f1);
            step(t + 1, f1, f0);
        }
        if (t + 1 < L) {                               // two slabs left
            step(t, f0, f1);
            f0 = f1;
        }
        Mode::template mma<FM, FN>(f0, acc);           // the last slab
    }

    // Epilogue: register r of lane l holds C[8(r/4) + 4(l/32) + r%4][l%32] of
    // each 32x32 block; 32 lanes write one 128-byte run of a row of C. C is
    // addressed as global memory: a generic (flat) access could alias LDS and
    // would have to wait for the direct loads still in flight.
    global_f32 *C = (global_f32 *)op.C;
    const global_i32 *row_exp = (const global_i32 *)op.row_exp;
    const global_i32 *col_exp = (const global_i32 *)op.col_exp;
    // The accumulate form reads a block's 16 values of C before any store, so
    // the loads are in flight together; the other forms have no trace of it.
    auto epilogue = [&](auto acc_form) {
        constexpr bool ACC = decltype(acc_form)::value;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int64_t j = j0 + wn * WN + b * 32 + (lane & 31);
                if (j >= op.p) continue;
                const int fj = Mode::SCALED && !partial ? col_exp[j] : 0;
                float old[16];
                if constexpr (ACC) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                        if (i < op.m) old[r] = C[i * op.p + j];
                    }
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t i = i0 + wm * WM + a * 32 + mfma32_row(r, lane);
                    if (i < op.m) {
                        float v = acc[a][b][r];
                        if (partial) {
                            ((global_f32 *)partial)[i * op.p + j] = v;
                            continue;
                        }
                        if constexpr (Mode::SCALED) v = ldexpf(v, -(row_exp[i] + fj));
                        if constexpr (ACC) v += old[r];
                        C[i * op.p + j] = v;
                    }
                }
            }
    };
    if (op.accumulate && !partial)
        epilogue(std::true_type{});
    else
        epilogue(std::false_type{});
}

// Tile-id -> block mapping of a single-product launch (XCD-aware bands).
__device__ __forceinline__ void block_of(int tiles_m, int tiles_n, int *tm, int *tn) {
    tile_coords(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
    // the integer divisions above run on the vector ALU; pin the (uniform)
    // results to scalar registers so everything derived from them stays scalar
    *tm = __builtin_amdgcn_readfirstlane(*tm);
    *tn = __builtin_amdgcn_readfirstlane(*tn);
}

// Workgroups per CU the register allocation must allow: two for four-wave
// blocks with a ring of more than 64 KiB that still leaves room for a second
// one in LDS (left to the compiler otherwise, which reaches three for the
// 48 KiB rings by itself).
template <int BM, int BN, int WM, int WN, int NREC, int NST>
constexpr int min_blocks() {
    using G = Cfg<BM, BN, WM, WN, NREC, NST>;
    return G::NW == 4 && G::LDS > 64 * 1024 && 2 * G::LDS <= 160 * 1024 ? 2 : 1;
}

template <int BM, int BN, int WM, int WN, int NREC, class Mode, int NST = NSTAGE>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, (min_blocks<BM, BN, WM, WN, NREC, NST>())) void single_kernel(Operands op, int tiles_m,
                                                                            int tiles_n) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[Cfg<BM, BN, WM, WN, NREC, NST>::LDS];
    int tm, tn;
    block_of(tiles_m, tiles_n, &tm, &tn);
    tile<BM, BN, WM, WN, NREC, Mode, NST>(op, (int64_t)tm * BM, (int64_t)tn * BN, lds);
}

// Split-k (the sigma loop cut into `chunks` contiguous runs of chunk_slabs
// slabs, Fig. 2's "addition loop" done across workgroups): workgroup w takes
// chunk w / tiles of tile w mod tiles (after the XCD remap, so the blocks of
// one chunk share an L2) and stores its raw block sum in partials + chunk m p.
template <int BM, int BN, int WM, int WN, int NREC, class Mode, int NST = NSTAGE>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void splitk_kernel(Operands op, int tiles_m, int tiles_n,
                                                                            int chunk_slabs, float *partials) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[Cfg<BM, BN, WM, WN, NREC, NST>::LDS];
    const int tiles = tiles_m * tiles_n;
    const int id = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, (int)gridDim.x));
    const int chunk = id / tiles;
    int tm, tn;
    tile_coords(id - chunk * tiles, tiles_m, tiles_n, 8, &tm, &tn);
    tm = __builtin_amdgcn_readfirstlane(tm);
    tn = __builtin_amdgcn_readfirstlane(tn);
    const int s_begin = chunk * chunk_slabs;
    const int s_end = min((int)op.S, s_begin + chunk_slabs);
    tile<BM, BN, WM, WN, NREC, Mode, NST>(op, (int64_t)tm * BM, (int64_t)tn * BN, lds, s_begin, s_end,
                                          partials + (int64_t)chunk * op.m * op.p);
}

// Deterministic reduction of the chunk partials: C = ((P_0 + P_1) + ...) + P_c-1,
// then the descale (scaled modes) and the accumulate form, as the epilogue of
// an unsplit product does.
static __global__ __launch_bounds__(256) void splitk_reduce_kernel(const float *__restrict__ partials, int chunks,
                                                            int64_t m, int64_t p, float *__restrict__ C,
                                                            const int32_t *__restrict__ row_exp,
                                                            const int32_t *__restrict__ col_exp, int accumulate) {
    const int64_t mp = m * p;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256) {
            const int64_t x = i * p + j;
            float v = partials[x];
            for (int q = 1; q < chunks; ++q) v += partials[(int64_t)q * mp + x];
            if (row_exp) v = ldexpf(v, -(row_exp[i] + col_exp[j]));
            if (accumulate) v += C[x];
            C[x] = v;
        }
}

// Host side of a split-k launch: chunk kernel, then the reduction.
template <int BM, int BN, int WM, int WN, int NREC, class Mode, int NST>
hipError_t launch_splitk(const Operands &op, int chunks, float *partials, hipStream_t st) {
    const int tiles_m = (int)((op.m + BM - 1) / BM), tiles_n = (int)((op.p + BN - 1) / BN);
    const int chunk_slabs = (int)((op.S + chunks - 1) / chunks);
    chunks = (int)((op.S + chunk_slabs - 1) / chunk_slabs);   // every chunk non-empty
    hipLaunchKernelGGL((splitk_kernel<BM, BN, WM, WN, NREC, Mode, NST>), dim3(tiles_m * tiles_n * chunks),
                       dim3(Cfg<BM, BN, WM, WN, NREC, NST>::THREADS), 0, st, op, tiles_m, tiles_n, chunk_slabs,
                       partials);
    const dim3 grid((unsigned)std::min<int64_t>((op.p + 255) / 256, 64), (unsigned)std::min<int64_t>(op.m, 65535));
    hipLaunchKernelGGL(splitk_reduce_kernel, grid, dim3(256), 0, st, partials, chunks, op.m, op.p, op.C, op.row_exp,
                       op.col_exp, op.accumulate);
    return hipGetLastError();
}

// Host check of the direct loads of single-product launches over an m x p
// product with S slabs and blocks of BM x BN (waves WM x WN, NREC record
// arrays per operand), through the same window functions as the kernel. For
// every block, wave and load: a live load's last window (slab S-1, where the
// offsets peak) lies inside its array's padded rows and inside its
// resource's range, with both offsets below 2^31; a dead load's tile lies
// wholly past the operand's padded rows (so its LDS rows feed only outputs
// that are not stored), and its vector offset 2^31 exceeds every resource
// range (num_records below 2^31). Returns the number of violations and the number of
// loads checked per slab in *loads.
inline int64_t check_loads(int BM, int BN, int WM, int WN, int NREC, int64_t m, int64_t p, int64_t S,
                           int64_t *loads) {
    const int NW = (BM / WM) * (BN / WN);
    const int ROWS = NREC * (BM + BN);
    const int LPW = ROWS / 16 / NW;
    const bool one_array = BM % (16 * LPW) == 0 && BN % (16 * LPW) == 0;
    const int64_t tile_row = S * GROUP * REC_BYTES;
    const int64_t lim31 = (int64_t(1) << 31) - 1;
    int64_t bad = 0, count = 0;
    if (ROWS % (16 * NW) != 0 || S <= 0) return 1;
    for (int64_t i0 = 0; i0 < m; i0 += BM)
        for (int64_t j0 = 0; j0 < p; j0 += BN)
            for (int wave = 0; wave < NW; ++wave) {
                const int row_first = wave * LPW * 16;
                const RowWindow w0 = row_window(BM, BN, NREC, row_first, i0, j0, m, p);
                const int q_split = q_split_of(BM, BN, NREC, LPW, one_array, row_first);
                const RowWindow w1 = q_split < LPW ? row_window(BM, BN, NREC, row_first + 16 * q_split, i0, j0, m, p) : w0;
                for (int q = 0; q < LPW; ++q) {
                    ++count;
                    const bool first = one_array || q < q_split;
                    const RowWindow &w = first ? w0 : w1;
                    const int tile_in = first ? w0.row_in / GROUP + q : w1.row_in / GROUP + (q - q_split);
                    // the load's rows in LDS must be the rows this window names
                    const RowWindow here = row_window(BM, BN, NREC, row_first + 16 * q, i0, j0, m, p);
                    if (here.a != w.a || here.arr != w.arr || here.row_in != tile_in * GROUP) ++bad;
                    const int64_t padded_tiles = padded_rows(w.a ? m : p) / GROUP;
                    const int64_t num_records = (int64_t)w.tiles * tile_row;
                    if (w.tiles < 1 || num_records > lim31) ++bad;
                    const int64_t soff = tile_in * tile_row + (S - 1) * GROUP * REC_BYTES;
                    if (soff > lim31) ++bad;
                    if (tile_in < w.tiles) {                  // live
                        const int64_t end = soff + GROUP * REC_BYTES;   // voffset < 1 KiB, 16 bytes each
                        if (w.first_tile + tile_in >= padded_tiles || end > num_records) ++bad;
                    } else if (w.first_tile + tile_in < padded_tiles) {
                        ++bad;                                // dead but inside the operand
                    }
                }
            }
    if (loads) *loads = count;
    return bad;
}

}  // namespace ring
}  // namespace moa
