// Plain ONF kernel: Eq. 3 with one fused multiply-add per (i, j, k), k in
// ascending order for every element of C.
//
// The paper's generic program walks row i of C and, for each k, adds the
// scalar A[i,k] times the contiguous row k of B (Fig. 1, section "From Normal
// Form to C Program"). Its dimension lifting (section "Dimension Lifting to
// Machine Coordinates") splits i over processors and j over register groups,
// and the k (sigma) loop into blocks. On gfx950 the same splits become:
//   i -> (workgroup row block of TM rows, lane row group; R rows per lane,
//         strided by the TR row groups of the workgroup)
//   j -> (workgroup column block of TN columns, lane column group; VJ columns
//         per lane in VJ/VW runs of VW contiguous elements = one 16-byte
//         vector each)
//   k -> (LDS slab of BK, in-slab index)
// Rows of A and B enter LDS as contiguous 16-byte vectors (coalesced row
// reads, the contiguous access Eq. 3 prescribes), double-buffered through
// registers. A column-major operand (the paper's gamma_col layout) is read
// along its contiguous extent and transposed on the way into the same
// row-major LDS slab, so the k loop below is the same for every layout. Each lane keeps its R x VJ block of C in registers for the whole
// k loop, so the k-sum of every element is the plain ascending sequence of
// fma(A[i,k], B[k,j], acc) -- bitwise the paper's loop with fma.
#include "moa_internal.h"
#include "ring_gemm.h"

namespace moa {
namespace {

template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int W = 2; };

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int TM, int TN, int BK, int R, int VJ>
__global__ __launch_bounds__(256) void onf_kernel(const T *__restrict__ A,
                                                  const T *__restrict__ B,
                                                  T *__restrict__ C, int64_t m,
                                                  int64_t n, int64_t p,
                                                  int accumulate, int vec_a,
                                                  int vec_b, int vec_c, int a_col,
                                                  int b_col) {
    using V = typename Vec<T>::type;
    constexpr int VW = Vec<T>::W;          // elements per 16-byte vector
    constexpr int TC = TN / VJ;            // lane column groups
    constexpr int TR = TM / R;             // lane row groups
    static_assert(TC * TR == 256, "256 threads");
    static_assert(VJ % VW == 0 && BK % VW == 0, "vector multiples");
    constexpr int G = VJ / VW;             // column runs per lane
    constexpr int PAD_A = VW;              // keeps rows 16-byte aligned, skews banks
    constexpr int LDA = BK + PAD_A;
    constexpr int A_VECS = TM * BK / VW;   // vectors per A slab
    constexpr int B_VECS = BK * TN / VW;
    constexpr int A_PER = (A_VECS + 255) / 256;
    constexpr int B_PER = (B_VECS + 255) / 256;

    __shared__ __attribute__((aligned(16))) T As[2][TM * LDA];
    __shared__ __attribute__((aligned(16))) T Bs[2][BK * TN];

    const int t = threadIdx.x;
    const int tr = t / TC;                 // row group
    const int tc = t % TC;                 // column group
    const int64_t i0 = (int64_t)blockIdx.y * TM;
    const int64_t j0 = (int64_t)blockIdx.x * TN;

    // ---- C block in registers; the accumulate form starts from C --------
    T acc[R][VJ];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int v = 0; v < VJ; ++v) acc[q][v] = T(0);
    if (accumulate) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t i = i0 + tr + (int64_t)TR * q;
            if (i >= m) continue;
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    const int64_t j = j0 + g * (TC * VW) + tc * VW + e;
                    if (j < p) acc[q][g * VW + e] = C[i * p + j];
                }
        }
    }

    // ---- global -> registers for one k slab ------------------------------
    V ra[A_PER], rb[B_PER];
    // whole blocks (inside m and p, the slab inside n, vector-aligned rows)
    // load without per-vector checks
    const bool inner = i0 + TM <= m && j0 + TN <= p && vec_a && vec_b && !a_col && !b_col;
    auto load_slab = [&](int64_t k0) {
        if (inner && k0 + BK <= n) {
#pragma unroll
            for (int s = 0; s < A_PER; ++s) {
                const int v = t + 256 * s;
                if (A_VECS % 256 == 0 || v < A_VECS)
                    ra[s] = *reinterpret_cast<const V *>(A + (i0 + v / (BK / VW)) * n + k0 + (v % (BK / VW)) * VW);
            }
#pragma unroll
            for (int s = 0; s < B_PER; ++s) {
                const int v = t + 256 * s;
                if (B_VECS % 256 == 0 || v < B_VECS)
                    rb[s] = *reinterpret_cast<const V *>(B + (k0 + v / (TN / VW)) * p + j0 + (v % (TN / VW)) * VW);
            }
            return;
        }
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int v = t + 256 * s;
            V val;
#pragma unroll
            for (int e = 0; e < VW; ++e) ((T *)&val)[e] = T(0);
            if (v < A_VECS && !a_col) {
                const int row = v / (BK / VW);
                const int kv = (v % (BK / VW)) * VW;
                const int64_t i = i0 + row, k = k0 + kv;
                if (i < m) {
                    if (vec_a && k + VW <= n) {
                        val = *reinterpret_cast<const V *>(A + i * n + k);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            if (k + e < n) ((T *)&val)[e] = A[i * n + k + e];
                    }
                }
            } else if (v < A_VECS) {
                // column-major A: element (i, k) at i + k m; a vector runs along i
                const int kk = v / (TM / VW);
                const int iv = (v % (TM / VW)) * VW;
                const int64_t i = i0 + iv, k = k0 + kk;
                if (k < n) {
                    if (vec_a && i + VW <= m) {
                        val = *reinterpret_cast<const V *>(A + k * m + i);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            if (i + e < m) ((T *)&val)[e] = A[k * m + i + e];
                    }
                }
            }
            ra[s] = val;
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int v = t + 256 * s;
            V val;
#pragma unroll
            for (int e = 0; e < VW; ++e) ((T *)&val)[e] = T(0);
            if (v < B_VECS && !b_col) {
                const int kk = v / (TN / VW);
                const int jv = (v % (TN / VW)) * VW;
                const int64_t k = k0 + kk, j = j0 + jv;
                if (k < n) {
                    if (vec_b && j + VW <= p) {
                        val = *reinterpret_cast<const V *>(B + k * p + j);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            if (j + e < p) ((T *)&val)[e] = B[k * p + j + e];
                    }
                }
            } else if (v < B_VECS) {
                // column-major B: element (k, j) at k + j n; a vector runs along k
                const int jj = v / (BK / VW);
                const int kv = (v % (BK / VW)) * VW;
                const int64_t j = j0 + jj, k = k0 + kv;
                if (j < p) {
                    if (vec_b && k + VW <= n) {
                        val = *reinterpret_cast<const V *>(B + j * n + k);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            if (k + e < n) ((T *)&val)[e] = B[j * n + k + e];
                    }
                }
            }
            rb[s] = val;
        }
    };
    auto store_slab = [&](int buf) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int v = t + 256 * s;
            if (v < A_VECS && !a_col) {
                const int row = v / (BK / VW);
                const int kv = (v % (BK / VW)) * VW;
                *reinterpret_cast<V *>(&As[buf][row * LDA + kv]) = ra[s];
            } else if (v < A_VECS) {           // transposed into the row-major slab
                const int kk = v / (TM / VW);
                const int iv = (v % (TM / VW)) * VW;
#pragma unroll
                for (int e = 0; e < VW; ++e) As[buf][(iv + e) * LDA + kk] = ((const T *)&ra[s])[e];
            }
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int v = t + 256 * s;
            if (v < B_VECS && !b_col) {
                const int kk = v / (TN / VW);
                const int jv = (v % (TN / VW)) * VW;
                *reinterpret_cast<V *>(&Bs[buf][kk * TN + jv]) = rb[s];
            } else if (v < B_VECS) {
                const int jj = v / (BK / VW);
                const int kv = (v % (BK / VW)) * VW;
#pragma unroll
                for (int e = 0; e < VW; ++e) Bs[buf][(kv + e) * TN + jj] = ((const T *)&rb[s])[e];
            }
        }
    };

    // ---- one in-slab step: k ascending ------------------------------------
    auto step = [&](const T *as, const T *bs, int kk) {
        T a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = as[(tr + TR * q) * LDA + kk];
        T b[VJ];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const V bv = *reinterpret_cast<const V *>(&bs[kk * TN + g * (TC * VW) + tc * VW]);
#pragma unroll
            for (int e = 0; e < VW; ++e) b[g * VW + e] = ((const T *)&bv)[e];
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int v = 0; v < VJ; ++v) acc[q][v] = fma_t(a[q], b[v], acc[q][v]);
    };

    const int64_t nslabs = (n + BK - 1) / BK;
    if (nslabs > 0) {
        load_slab(0);
        store_slab(0);
        __syncthreads();
    }
    for (int64_t s = 0; s < nslabs; ++s) {
        const int buf = (int)(s & 1);
        const int64_t k0 = s * BK;
        if (s + 1 < nslabs) load_slab(k0 + BK);
        const T *as = As[buf];
        const T *bs = Bs[buf];
        const int64_t kn = n - k0;
        if (kn >= BK) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += VW) {
                // A values for VW consecutive k come from one vector read per row
                V av[R];
#pragma unroll
                for (int q = 0; q < R; ++q)
                    av[q] = *reinterpret_cast<const V *>(&as[(tr + TR * q) * LDA + kk]);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    T b[VJ];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const V bv = *reinterpret_cast<const V *>(
                            &bs[(kk + e) * TN + g * (TC * VW) + tc * VW]);
#pragma unroll
                        for (int w = 0; w < VW; ++w) b[g * VW + w] = ((const T *)&bv)[w];
                    }
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const T a = ((const T *)&av[q])[e];
#pragma unroll
                        for (int v = 0; v < VJ; ++v) acc[q][v] = fma_t(a, b[v], acc[q][v]);
                    }
                }
            }
        } else {
            for (int kk = 0; kk < (int)kn; ++kk) step(as, bs, kk);
        }
        if (s + 1 < nslabs) store_slab(buf ^ 1);
        __syncthreads();
    }

    // ---- write the C block: contiguous runs of row i ----------------------
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t i = i0 + tr + (int64_t)TR * q;
        if (i >= m) continue;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t j = j0 + g * (TC * VW) + tc * VW;
            if (vec_c && j + VW <= p) {
                V out;
#pragma unroll
                for (int e = 0; e < VW; ++e) ((T *)&out)[e] = acc[q][g * VW + e];
                *reinterpret_cast<V *>(C + i * p + j) = out;
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    if (j + e < p) C[i * p + j + e] = acc[q][g * VW + e];
            }
        }
    }
}

// ONF on a direct-load LDS ring. A slab is one 64-byte row of A per row of
// the block (BK = 8 doubles or 16 floats of k) and the matching BK rows of B;
// the slabs go from memory straight into LDS (`buffer_load ... lds`), so no
// registers hold them in flight and a lane can keep a large block of C:
// 128 x 128 blocks, 8 x 8 per lane (8 + 8 elements of LDS per k for 64
// FMAs: 2 bytes per FMA in FP64, which the LDS delivers at the FP64 FMA rate,
// 1 byte in FP32; a 16 x 8 FP32 lane block would need more than 256
// registers). Per slab:
//   A: TM rows of 64 bytes, 16-byte chunk c of row r at physical chunk
//      c ^ ((r / 4) mod 4) (conflict-free reads by rows of lanes);
//   B: the slab's BK rows of TN elements, contiguous.
// Lane (tr, tc) owns rows tr + TR q of the block and, for each 16-byte chunk
// g of its columns, elements (g TC + tc) (16 / size) + u. Rows past m and
// slab rows past n read as zeros (buffer ranges); columns past p are never
// stored. The k loop is the same ascending fma sequence per element as the
// register-staged kernel, and the last slab stops at n (no padded steps), so
// results are bitwise the same.
// Ring depth and workgroups per CU: FP32 three 16 KiB stages and three
// workgroups per CU (the kernel fits 128 VGPRs), FP64 four stages and two
// (its 64 FP64 accumulators per lane would spill at three).
constexpr int ONF64_NST = 4, ONF32_NST = 3;
template <typename T> constexpr int ring_occupancy() { return sizeof(T) == 4 ? 3 : 2; }

// N elements of T as one vector register value
template <typename T, int N> struct ExtVec { typedef T type __attribute__((ext_vector_type(N))); };

template <typename T, int TM, int TN, int R, int VJ, int NST>
__device__ __forceinline__ void onf_ring_block(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ C,
                                               int64_t m, int64_t n, int64_t p, int accumulate, int vec_c,
                                               uint8_t *lds) {
    constexpr int ES = (int)sizeof(T), BK = 64 / ES, EPC = 16 / ES;   // k per slab, elements per 16-byte chunk
    constexpr int TR = TM / R, TC = TN / VJ, GC = VJ / EPC;           // lane rows, lane columns, chunks per lane
    constexpr int A_BYTES = TM * 64, B_BYTES = BK * TN * ES, STAGE = A_BYTES + B_BYTES;
    constexpr int LPW = STAGE / 1024 / 4;                                // KiB loads per wave per slab
    constexpr int RPL = 1024 / (TN * ES), CPR = TN * ES / 16;           // B rows per load, chunks per B row
    static_assert(TR * TC == 256 && STAGE % 4096 == 0 && VJ % EPC == 0 && RPL >= 1, "shape of the ONF ring");
    static_assert(NST >= 3 && NST <= 4, "waits cover up to two later slabs");
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int tr = t / TC, tc = t % TC;
    const int64_t i0 = (int64_t)blockIdx.y * TM, j0 = (int64_t)blockIdx.x * TN;
    auto col = [&](int v) { return (v / EPC * TC + tc) * EPC + v % EPC; };   // lane column v in the block

    // the accumulate form starts from C
    T acc[R][VJ];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int v = 0; v < VJ; ++v) acc[q][v] = T(0);
    if (accumulate) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t i = i0 + tr + TR * q;
            if (i >= m) continue;
#pragma unroll
            for (int v = 0; v < VJ; ++v) {
                const int64_t j = j0 + col(v);
                if (j < p) acc[q][v] = C[i * p + j];
            }
        }
    }

    const int64_t rows_live = m - i0 < TM ? m - i0 : TM;
    const int64_t a_range = rows_live * n * ES;
    const int64_t b_total = n * p - j0;        // elements from B + j0 to the end of B
    const int64_t S = (n + BK - 1) / BK;

    // Both resources start at the slab (A: column k0 of the block's first
    // row, B: row k0) and end where the live data ends, so each lane's vector
    // offset is the same for every slab: computed once, in registers no later
    // instruction overwrites.
    int voff[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int g = wave * LPW + q;                     // wave-uniform
        if (g < A_BYTES / 1024) {
            const int r = 16 * g + (lane >> 2);
            const int c = (lane & 3) ^ ((lane >> 4) & 3);
            voff[q] = r < rows_live ? (int)(((int64_t)r * n + EPC * c) * ES) : ring::kDeadVoffset;
        } else {
            const int row = (g - A_BYTES / 1024) * RPL + lane / CPR;
            voff[q] = (int)(((int64_t)row * p + EPC * (lane % CPR)) * ES);
        }
    }
    auto issue_to = [&](uint8_t *buf, int64_t s) {     // buf: stage s mod NST
        const int64_t k0 = s * BK;
        const int64_t a_left = a_range - k0 * ES, b_left = (b_total - k0 * p) * ES;
        const __amdgpu_buffer_rsrc_t a_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + i0 * n + k0), (short)0, (int)(a_left > 0 ? a_left : 0), 0x00020000);
        const __amdgpu_buffer_rsrc_t b_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B + j0 + k0 * p), (short)0, (int)(b_left < 0x7FFFFFFF ? b_left : 0x7FFFFFFF), 0x00020000);
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int g = wave * LPW + q;
            if (g < A_BYTES / 1024)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(a_rsrc, (ring::lds_void_t *)(buf + g * 1024), 16, voff[q], 0,
                                                         0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    b_rsrc, (ring::lds_void_t *)(buf + A_BYTES + (g - A_BYTES / 1024) * 1024), 16, voff[q], 0, 0, 0);
        }
    };

    // the 16-byte chunk of A row r holding k .. k + EPC - 1 (k a multiple of EPC)
    using chunk_t = typename ExtVec<T, EPC>::type;
    auto a_chunk = [&](const uint8_t *buf, int r, int k) {
        return *reinterpret_cast<const chunk_t *>(buf + r * 64 + (((k / EPC) ^ ((r >> 2) & 3)) << 4));
    };
    // a lane's VJ elements of B row k
    auto b_row = [&](const uint8_t *bs, int k, T (&b)[VJ]) {
#pragma unroll
        for (int g = 0; g < GC; ++g) {
            const chunk_t v = *reinterpret_cast<const chunk_t *>(bs + k * TN * ES + (g * TC + tc) * 16);
#pragma unroll
            for (int u = 0; u < EPC; ++u) b[g * EPC + u] = v[u];
        }
    };

    // one whole slab (BK k, ascending) from `buf`
    auto compute_full = [&](const uint8_t *buf) {
        const uint8_t *bs = buf + A_BYTES;
#pragma unroll
        for (int kk = 0; kk < BK; kk += EPC) {
            chunk_t av[R];
#pragma unroll
            for (int q = 0; q < R; ++q) av[q] = a_chunk(buf, tr + TR * q, kk);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                T b[VJ];
                b_row(bs, kk + e, b);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const T a = av[q][e];
#pragma unroll
                    for (int v = 0; v < VJ; ++v) acc[q][v] = fma_t(a, b[v], acc[q][v]);
                }
            }
        }
    };
    // the last, partial slab: k values 0 .. kc - 1 only (no padded steps)
    auto compute_tail = [&](const uint8_t *buf, int kc) {
        const uint8_t *bs = buf + A_BYTES;
        for (int kk = 0; kk < kc; ++kk) {
            T a[R], b[VJ];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const chunk_t c = a_chunk(buf, tr + TR * q, kk - kk % EPC);
                a[q] = c[kk % EPC];
            }
            b_row(bs, kk, b);
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int v = 0; v < VJ; ++v) acc[q][v] = fma_t(a[q], b[v], acc[q][v]);
        }
    };

    // One step: the stage the step's loads fill (slab s + NST - 1) and the
    // stage it computes (slab s) are disjoint LDS, passed as restrict
    // pointers so that the compiler sees the reads need not wait for those
    // loads, which are meant to stay in flight (the explicit wait before the
    // barrier orders slab s's own loads).
    auto step = [&](uint8_t *__restrict__ dma, const uint8_t *__restrict__ cur, int64_t s) {
        if (s + NST - 1 < S) issue_to(dma, s + NST - 1);
        compute_full(cur);
    };
    // Per slab: slab s has landed in every wave and every wave is done with
    // slab s - 1, whose stage slab s + NST - 1 then takes.
    const int64_t full = n / BK;
    for (int q = 0; q < NST - 1; ++q)
        if (q < S) issue_to(lds + q * STAGE, q);
    for (int64_t s = 0; s < full; ++s) {
        // slab s landed; at most NST - 2 later slabs of this wave in flight
        const int64_t ahead = S - 1 - s < NST - 2 ? S - 1 - s : NST - 2;
        if (ahead >= 2) __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(2 * LPW));
        else if (ahead == 1) __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(LPW));
        else __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(0));
        ring::ring_barrier();
        step(lds + ((s + NST - 1) % NST) * STAGE, lds + (s % NST) * STAGE, s);
    }
    if (full < S) {
        __builtin_amdgcn_s_waitcnt(ring::waitcnt_vm(0));
        ring::ring_barrier();
        compute_tail(lds + (full % NST) * STAGE, (int)(n - full * BK));
    }

#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t i = i0 + tr + TR * q;
        if (i >= m) continue;
#pragma unroll
        for (int g = 0; g < GC; ++g) {
            const int64_t j = j0 + (g * TC + tc) * EPC;
            if (vec_c && j + EPC <= p) {
                chunk_t v;
#pragma unroll
                for (int u = 0; u < EPC; ++u) v[u] = acc[q][g * EPC + u];
                *reinterpret_cast<chunk_t *>(C + i * p + j) = v;
            } else {
#pragma unroll
                for (int u = 0; u < EPC; ++u)
                    if (j + u < p) C[i * p + j + u] = acc[q][g * EPC + u];
            }
        }
    }
}

template <typename T, int TM, int TN, int R, int VJ, int NST>
__global__ __launch_bounds__(256, ring_occupancy<T>()) void onf_ring_kernel(const T *__restrict__ A, const T *__restrict__ B,
                                                         T *__restrict__ C, int64_t m, int64_t n, int64_t p,
                                                         int accumulate, int vec_c) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[NST * (TM * 64 + 64 / sizeof(T) * TN * sizeof(T))];
    onf_ring_block<T, TM, TN, R, VJ, NST>(A, B, C, m, n, p, accumulate, vec_c, lds);
}

template <typename T, int TM, int TN, int R, int VJ, int NST>
hipError_t launch_ring(const moa_gemm_desc &d, hipStream_t st) {
    const T *A = static_cast<const T *>(d.A);
    const T *B = static_cast<const T *>(d.B);
    T *C = static_cast<T *>(d.C);
    const int vec_c = (d.p % (16 / (int)sizeof(T)) == 0) && ((uintptr_t)C % 16 == 0);
    dim3 grid((unsigned)((d.p + TN - 1) / TN), (unsigned)((d.m + TM - 1) / TM));
    hipLaunchKernelGGL((onf_ring_kernel<T, TM, TN, R, VJ, NST>), grid, dim3(256), 0, st, A, B, C, d.m, d.n, d.p,
                       d.accumulate, vec_c);
    return hipGetLastError();
}

struct OnfShape { int tm, tn, bk, r, vj; };

// Instantiation tables. The first entry per type is the paper's static block
// for the 32 KB vector L1 (three blocks of A, B and C): 1024 FP64 components
// (32 x 32) and 2048 FP32 components (32 x 64). Larger entries trade LDS for
// register blocking; the planner picks among them.
// The last entry per type is the direct-load ring kernel above (row-major
// operands).
constexpr OnfShape kF64[] = {{32, 32, 16, 2, 2}, {64, 64, 16, 4, 4}, {64, 128, 16, 4, 8}, {128, 128, 16, 8, 8},
                             {128, 128, 8, 8, 8}};
constexpr OnfShape kF32[] = {{32, 64, 16, 2, 4}, {64, 64, 16, 4, 4}, {64, 128, 16, 4, 8}, {128, 128, 16, 8, 8},
                             {128, 128, 16, 8, 8}};

template <typename T, int TM, int TN, int BK, int R, int VJ>
hipError_t launch_one(const moa_gemm_desc &d, hipStream_t st) {
    const T *A = static_cast<const T *>(d.A);
    const T *B = static_cast<const T *>(d.B);
    T *C = static_cast<T *>(d.C);
    constexpr int VW = Vec<T>::W;
    const int a_col = (d.flags & MOA_FLAG_A_COL) != 0, b_col = (d.flags & MOA_FLAG_B_COL) != 0;
    // 16-byte vectors run along the contiguous extent of each operand
    const int vec_a = ((a_col ? d.m : d.n) % VW == 0) && ((uintptr_t)A % 16 == 0);
    const int vec_b = ((b_col ? d.n : d.p) % VW == 0) && ((uintptr_t)B % 16 == 0);
    const int vec_c = (d.p % VW == 0) && ((uintptr_t)C % 16 == 0);
    dim3 grid((unsigned)((d.p + TN - 1) / TN), (unsigned)((d.m + TM - 1) / TM));
    hipLaunchKernelGGL((onf_kernel<T, TM, TN, BK, R, VJ>), grid, dim3(256), 0, st, A, B, C,
                       d.m, d.n, d.p, d.accumulate, vec_a, vec_b, vec_c, a_col, b_col);
    return hipGetLastError();
}

}  // namespace

int onf_variant_count(moa_dtype t) {
    return t == MOA_F64 ? (int)(sizeof(kF64) / sizeof(kF64[0]))
                        : (int)(sizeof(kF32) / sizeof(kF32[0]));
}

void onf_variant_shape(moa_dtype t, int v, Plan *p) {
    const OnfShape s = (t == MOA_F64) ? kF64[v] : kF32[v];
    const int es = (t == MOA_F64) ? 8 : 4;
    p->variant = v;
    p->tile_m = s.tm;
    p->tile_n = s.tn;
    p->tile_k = s.bk;
    p->lane_m = s.r;
    p->lane_n = s.vj;
    p->wave_m = s.r * (64 / (s.tn / s.vj));
    p->wave_n = s.tn;
    p->threads = 256;
    p->lds_bytes = 2 * (s.tm * (s.bk + 16 / es) + s.bk * s.tn) * es;
    if (v == onf_ring_variant(t)) p->lds_bytes = (t == MOA_F64 ? ONF64_NST : ONF32_NST) * (s.tm + s.tn) * s.bk * es;
}

int onf_ring_variant(moa_dtype t) { return onf_variant_count(t) - 1; }

// The ring kernel's 32-bit buffer offsets: 130 rows of n elements of A,
// BK + 1 rows of p elements of B (BK 8 in FP64, 16 in FP32).
bool onf_ring_fits(moa_dtype t, int64_t n, int64_t p) {
    return t == MOA_F64 ? 130 * n * 8 < 0x7FFFFFFF && 9 * p * 8 < 0x7FFFFFFF
                        : 130 * n * 4 < 0x7FFFFFFF && 17 * p * 4 < 0x7FFFFFFF;
}

hipError_t launch_onf(const moa_gemm_desc &d, const Plan &plan, hipStream_t st) {
    if (d.dtype == MOA_F64) {
        switch (plan.variant) {
        case 0: return launch_one<double, 32, 32, 16, 2, 2>(d, st);
        case 1: return launch_one<double, 64, 64, 16, 4, 4>(d, st);
        case 2: return launch_one<double, 64, 128, 16, 4, 8>(d, st);
        case 3: return launch_one<double, 128, 128, 16, 8, 8>(d, st);
        default: return launch_ring<double, 128, 128, 8, 8, ONF64_NST>(d, st);
        }
    }
    switch (plan.variant) {
    case 0: return launch_one<float, 32, 64, 16, 2, 4>(d, st);
    case 1: return launch_one<float, 64, 64, 16, 4, 4>(d, st);
    case 2: return launch_one<float, 64, 128, 16, 4, 8>(d, st);
    case 3: return launch_one<float, 128, 128, 16, 8, 8>(d, st);
    default: return launch_ring<float, 128, 128, 8, 8, ONF32_NST>(d, st);
    }
}

}  // namespace moa
