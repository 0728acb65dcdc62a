/*
 * moa.h -- C ABI of the MoA ONF matrix-product library for AMD Instinct
 * MI355X (gfx950 / CDNA4).
 *
 * The operation (Mullin, "From array algebra to energy efficiency on GPUs",
 * section "MoA Matrix Multiplication", Eq. 1-3): with shapes
 *     rho A = <m, n>,  rho B = <n, p>,  rho C = <m, p>
 * and all three arrays stored row-major and contiguous from their base
 * addresses (the address form that follows Eq. 3; no strides, no padding),
 *     C[i*p + j] := sum_{k=0}^{n-1} A[i*n + k] * B[k*p + j]
 * for 0 <= i < m, 0 <= j < p (index bounds of Eq. 2). The paper's generic C
 * program adds into C instead of assigning; `accumulate != 0` selects that
 * form (C += A.B), `accumulate == 0` the assignment of Eq. 3.
 *
 * Conventions for every call below:
 *  - Sizes are int64_t and may exceed 2^31 elements. m, n or p may be 0:
 *    n == 0 is the empty sum (C := 0, or C unchanged when accumulating);
 *    m == 0 or p == 0 writes nothing.
 *  - Matrix pointers are DEVICE pointers on the current HIP device, owned by
 *    the caller, aligned to at least the element size; 16-byte alignment is
 *    recommended (other alignments are accepted). The library never frees
 *    them; they must stay valid until the work on `stream` has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on it unless stated otherwise.
 *  - Argument errors are returned synchronously and nothing is launched.
 *    A failed launch returns MOA_ERR_DEVICE. No C++ exception crosses the
 *    ABI. moa_last_error() gives a thread-local message for the last error.
 *  - Calls on different streams may run concurrently; each call uses only
 *    its own arguments and, where it needs scratch space, a device buffer
 *    of the library's cache that no unfinished work on another stream still
 *    uses (the stream-ordered allocator while the stream is being captured).
 *    A buffer last used on the calling stream is reused at once (stream
 *    order covers the earlier use), so synchronize a stream before
 *    destroying it: a new stream that receives the same handle would
 *    otherwise not be ordered after the old stream's pending calls.
 *    The cache keeps buffers between calls (at most 64 GiB per device); the
 *    serving loop does not use it (its scratch comes from its budgeted
 *    pool).
 */
#ifndef MOA_H
#define MOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum moa_status {
    MOA_OK = 0,
    MOA_ERR_INVALID = 1,      /* null pointer, bad enum, aliasing, bad count */
    MOA_ERR_SHAPE = 2,        /* negative size or size overflow */
    MOA_ERR_UNSUPPORTED = 3,  /* dtype/path combination not provided */
    MOA_ERR_NOMEM = 4,        /* scratch allocation failed / over budget */
    MOA_ERR_DEVICE = 5,       /* HIP error from a launch or runtime call */
    MOA_NOT_READY = 6         /* serving: request not finished yet */
} moa_status;

typedef enum moa_dtype {
    MOA_F64 = 0,              /* double A, B, C */
    MOA_F32 = 1               /* float A, B, C */
} moa_dtype;

/* How the contraction is carried out. Every path computes Eq. 3; they
 * differ in arithmetic:
 *  ONF          -- scalar fused multiply-add, k ascending for every element
 *                  (the paper's loop order); FP64 or FP32. Bitwise equal to
 *                  the same loop with one fma per step.
 *  MFMA_F32     -- FP32 matrix-core tiles (v_mfma_f32_32x32x2_f32), FP32
 *                  accumulation. F32 only. Variants 0, 1 copy A's rows and
 *                  B's columns into 64-byte records (scratch of 4 (m + p) n
 *                  bytes, n <= 16 * 131071) and run the record ring;
 *                  variant 2 stages through registers and takes no scratch.
 *  SPLIT_BF16   -- each FP32 input x is split into hi = RNE_bf16(x) and
 *                  lo = RNE_bf16(x - hi); C = hi.hi + hi.lo + lo.hi on BF16
 *                  matrix cores with FP32 accumulation. F32 only.
 *  FP8_SCALED   -- row i of A is scaled by 2^e_i and column j of B by 2^f_j
 *                  (e the largest integer with amax * 2^e <= 448), rounded
 *                  to OCP E4M3, multiplied on FP8 matrix cores with FP32
 *                  accumulation and descaled exactly by 2^-(e_i+f_j).
 *                  By default the rounding residual is kept as a second
 *                  E4M3 term (stored times 2^4) and
 *                  C = 2^-(e_i+f_j) (h.h + 2^-4 (h.l + l.h)); with
 *                  MOA_FLAG_FP8_ONE_TERM only h.h is formed. F32 only.
 *  AUTO         -- ONF for F64, SPLIT_BF16 for F32.
 * The split and FP8 paths require finite inputs. */
typedef enum moa_path {
    MOA_PATH_AUTO = 0,
    MOA_PATH_ONF = 1,
    MOA_PATH_MFMA_F32 = 2,
    MOA_PATH_SPLIT_BF16 = 3,
    MOA_PATH_FP8_SCALED = 4
} moa_path;

/* Term count of the scaled-FP8 path. Two terms are the default (normwise
 * error about 1e-3 against Eq. 3 on rows and columns spanning 10^+-3, within
 * the 3e-2 bar of that path); MOA_FLAG_FP8_TWO_TERM names the default
 * explicitly. MOA_FLAG_FP8_ONE_TERM opts into the single E4M3 term: about
 * four times faster, but its error is about 3.7e-2 -- the four significant
 * bits of E4M3, which no power-of-two scale improves -- above that bar.
 * Setting both is MOA_ERR_INVALID. */
#define MOA_FLAG_FP8_TWO_TERM 0x1u
#define MOA_FLAG_FP8_ONE_TERM 0x2u
/* Forces instantiation `v` (0-based) of the path's kernel table instead of
 * the planner's choice: the block sizes of the dimension lift, for block-size
 * sweeps and autotuning (moa_plan_query reports the resulting shape). An
 * index beyond the table is MOA_ERR_INVALID. Occupies flag bits 8..15. */
#define MOA_FLAG_VARIANT(v) ((uint32_t)((v) + 1) << 8)
#define MOA_FLAG_VARIANT_MASK 0xFF00u
/* Split-k, the sigma-lift of Fig. 2 carried across workgroups (its "addition
 * loop" over k blocks): the k slabs are cut into `c` contiguous chunks
 * (2 <= c <= 255; clamped so that no chunk is empty), each workgroup sums one
 * chunk of one block of C into an FP32 partial, and a second kernel adds the
 * partials in chunk order, then applies the FP8 descale and the accumulate
 * form. For products with fewer blocks of C than compute units and a long k
 * walk. Split-BF16 and FP8 paths only (MOA_ERR_UNSUPPORTED otherwise).
 * Without the flag the planner splits by itself when the product's 128 x 128
 * blocks number at most 64 and n >= 4096 (about 512 workgroups, chunks of at
 * least 512 k); MOA_FLAG_SPLIT_K(1) keeps such a product unsplit. The result
 * is deterministic and within the path's error bound, but its summation order
 * differs from the unsplit product's, so it is not bitwise equal to it.
 * Grouped launches and the serving loop run split members as single launches
 * (the same plan as alone, so the same result); prepared groups refuse them.
 * The partials (c m p FP32 values) are part of the workspace. Occupies flag
 * bits 16..23. */
#define MOA_FLAG_SPLIT_K(c) (((uint32_t)(c) & 0xFFu) << 16)
#define MOA_FLAG_SPLIT_K_MASK 0xFF0000u
/* Operand layouts from the paper's family of layout functions gamma (gamma_row,
 * the default, and gamma_col; conclusion and appendix): with MOA_FLAG_A_COL
 * the m x n matrix A is stored column by column, element (i, k) at offset
 * i + k m; MOA_FLAG_B_COL likewise stores B (n x p) as k + j n and
 * MOA_FLAG_C_COL stores C (m x p) as i + j m. Shapes keep their meaning.
 * Every path takes any combination; a column-major C is computed as
 * C^T = B^T A^T with a row-major result (no copies). The split-BF16, FP8 and
 * FP32 matrix-core ring paths condition a column-major operand with the other
 * packer; the ONF kernel reads it along its contiguous extent and transposes
 * it into its LDS slab, its k loop unchanged (bitwise the same result). The
 * register-staged FP32 variant (MOA_FLAG_VARIANT(2)) takes row-major operands
 * only (MOA_ERR_UNSUPPORTED otherwise). Grouped launches run members with a
 * column-major operand singly; prepared groups refuse them. */
#define MOA_FLAG_A_COL 0x1000000u
#define MOA_FLAG_B_COL 0x2000000u
#define MOA_FLAG_C_COL 0x4000000u
#define MOA_FLAG_LAYOUT_MASK 0x7000000u

/* One matrix product. Field names follow Eq. 1: m rows of A and C, n the
 * shared extent (rho B[0]), p columns of B and C. */
typedef struct moa_gemm_desc {
    int64_t m, n, p;
    int32_t dtype;            /* moa_dtype */
    int32_t path;             /* moa_path */
    const void *A;            /* device, m*n elements, row-major */
    const void *B;            /* device, n*p elements, row-major */
    void *C;                  /* device, m*p elements, row-major; must not
                                 overlap A or B */
    int32_t accumulate;       /* 0: C := A.B (Eq. 3); else C += A.B */
    uint32_t flags;           /* MOA_FLAG_* */
} moa_gemm_desc;

/* The dimension lift chosen for a product: how i, j and k are split over
 * workgroups, waves, lanes and LDS slabs (section "Dimension Lifting to
 * Machine Coordinates"), plus the paper's static block size for the type. */
typedef struct moa_plan_info {
    int32_t path;             /* resolved moa_path */
    int32_t kernel;           /* internal kernel id (for reports) */
    int32_t tile_m, tile_n;   /* C block per workgroup (rows x cols) */
    int32_t tile_k;           /* k slab staged in LDS per step */
    int32_t wave_m, wave_n;   /* C block per wavefront */
    int32_t lane_m, lane_n;   /* C block per lane (ONF) or 0 (matrix cores) */
    int32_t threads;          /* threads per workgroup */
    int32_t lds_bytes;        /* LDS per workgroup */
    int64_t workgroups;       /* grid size */
    int64_t workspace_bytes;  /* scratch taken from the stream allocator */
    int64_t static_components;/* static block size rule result (components) */
    int32_t variant;          /* instantiation of the path's kernel table */
    int32_t tuned;            /* 1 if the variant came from the autotuner */
    int32_t split_k;          /* k chunks summed by separate workgroups (1 = none) */
    int32_t reserved;
} moa_plan_info;

/* Eq. 3 on the device. Asynchronous on `stream`.
 * Errors: MOA_ERR_INVALID (null desc/pointers with non-empty sizes, C
 * overlapping A or B, unknown enum or flag), MOA_ERR_SHAPE (negative size,
 * element count overflow), MOA_ERR_UNSUPPORTED (F64 with a matrix-core path),
 * MOA_ERR_NOMEM (scratch), MOA_ERR_DEVICE (launch failure). */
moa_status moa_gemm(const moa_gemm_desc *desc, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the product of
 * moa_gemm -- same plan, same kernels, bitwise the same C -- with every
 * scratch buffer (conditioned record tiles, exponents, split-k partials)
 * placed in one fixed array of MOA_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds per GPU from the first call on that GPU until the process
 * ends. The call allocates and frees nothing and records no memset; the
 * caller still owns A, B and C. Every call on one GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (on
 * different streams without ordering) race and give undefined results;
 * calls ordered on one stream do not. Errors: as moa_gemm; MOA_ERR_NOMEM,
 * with nothing launched, if the product needs more scratch than the array
 * holds (moa_plan_info::workspace_bytes reports the need); the ONF path
 * needs none. */
#define MOA_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
moa_status moa_gemm_noalloc(const moa_gemm_desc *desc, void *stream);

/* `count` independent products (the blocked inner product of Fig. 2 over
 * many products at once). Row-major members on the split-BF16 path
 * (including F32 with MOA_PATH_AUTO) are contracted by ONE persistent launch
 * that walks a shared tile list and splits the FP32 operands into hi/lo BF16
 * on the way through LDS (no conditioning pass); scaled-FP8 members are
 * conditioned together and contracted by one persistent launch per term
 * count; members on the ONF and FP32 matrix-core paths, and members with a
 * column-major operand or a split k walk, run as single launches on the same
 * stream. No ordering among members. Each result is bitwise the result
 * moa_gemm gives for the same descriptor, whichever persistent kernel runs.
 * Descriptors are read on the host during the call; the array may be reused
 * when the call returns.
 * Errors: as moa_gemm, checked for every member before anything launches;
 * MOA_ERR_INVALID for count < 0, a null array with count > 0, or a member's
 * C overlapping any member's A, B or C. */
moa_status moa_gemm_grouped(const moa_gemm_desc *descs, int64_t count,
                            void *stream);

/* The persistent split-BF16 kernel of a grouped launch (the dimension lift of
 * section "Dimension Lifting to Machine Coordinates" applied to a work list
 * of blocks from many products):
 *   0  128 x 128 blocks, each slab split once into one LDS plane set, three
 *      workgroups per CU;
 *   1  128 x 128, two plane sets and a deeper ring, two per CU;
 *   2  128 x 128, split in registers by every wave that reads a fragment,
 *      two per CU;
 *   3  64 x 128 blocks, split once, four per CU;
 *   4  128 x 64 blocks, split once, four per CU.
 * moa_gemm_grouped and moa_group_create use the autotuner's record for the
 * members' class if there is one, else the static rule: the block among 2, 3
 * and 4 with the fewest slab steps over the members, weighted by the
 * measured time of one slab step of that block. moa_gemm_grouped_variant runs
 * moa_gemm_grouped with `variant` forced (-1: that choice); MOA_ERR_INVALID
 * for a variant outside -1 .. 4. */
#define MOA_GROUPED_VARIANTS 5
moa_status moa_gemm_grouped_variant(const moa_gemm_desc *descs, int64_t count, int32_t variant, void *stream);

/* The persistent split-BF16 kernel moa_gemm_grouped would use for these
 * members (no launch): `variant` (-1 when no member runs in it), `tuned` 1 if
 * it came from the autotuner, `persistent_members` the number of members in
 * that launch. Any output may be null. Errors: as moa_gemm_grouped. */
moa_status moa_grouped_plan_query(const moa_gemm_desc *descs, int64_t count, int32_t *variant, int32_t *tuned,
                                  int64_t *persistent_members);

/* Grouped autotuner: runs the whole grouped launch with each persistent
 * kernel in turn (one warm-up, then `reps` timed runs each, on `stream`,
 * overwriting every C), waits, and records the fastest for the class of the
 * persistent members -- ceil(log2) of their count and of their median m, n
 * and p -- which later grouped launches and prepared groups of that class
 * then use. The record is saved and loaded with the single-product records
 * (moa_autotune_save / _load) and cleared with them. `chosen` / `best_ms`
 * (may be null) receive the winner and its time per launch. Errors: as
 * moa_gemm_grouped; MOA_ERR_INVALID for reps < 1; MOA_ERR_UNSUPPORTED when no
 * member runs in the persistent split-BF16 launch. */
moa_status moa_autotune_grouped(const moa_gemm_desc *descs, int64_t count, int32_t reps, void *stream,
                                int32_t *chosen, double *best_ms);

/* The ipophp family (conclusion and appendix: the Hadamard, Kronecker and
 * matrix products in one formulation, higher-dimensional contractions as
 * many parallel 2-d products). A, B, C are row-major device arrays of
 * `dtype` (MOA_F32 or MOA_F64), asynchronous on `stream`. Each element is one
 * product rounded to the element type; with `accumulate` the rounded product
 * is added to C with a second rounding (no fused multiply-add), so results
 * are bitwise those of the definitions.
 *
 * Hadamard: C[i][j] := A[i][j] B[i][j] for m x n arrays. C may be A or B
 * itself (in place) but must not overlap them otherwise (MOA_ERR_INVALID).
 * Errors: MOA_ERR_SHAPE (negative or overflowing size), MOA_ERR_INVALID (null
 * pointer with a non-empty shape, unknown dtype, misalignment). */
moa_status moa_hadamard(int64_t m, int64_t n, int32_t dtype, const void *A, const void *B, void *C,
                        int32_t accumulate, void *stream);

/* Kronecker: A m x n, B p x q, C (m p) x (n q) with
 * C[i p + k][j q + l] := A[i][j] B[k][l]. C must not overlap A or B; n q must
 * stay below 2^31 (MOA_ERR_SHAPE). Errors as moa_hadamard. */
moa_status moa_kronecker(int64_t m, int64_t n, int64_t p, int64_t q, int32_t dtype, const void *A,
                         const void *B, void *C, int32_t accumulate, void *stream);

/* Batched products C[b] := A[b] B[b], b = 0 .. batch-1 (the 3-d contraction
 * as parallel 2-d products): member b is *first with A, B, C advanced by
 * b stride_a, b stride_b, b stride_c elements. Runs as moa_gemm_grouped over
 * the members (one persistent launch per path), with its checks and errors;
 * MOA_ERR_INVALID for a negative batch or stride. */
moa_status moa_gemm_batched(const moa_gemm_desc *first, int64_t batch, int64_t stride_a, int64_t stride_b,
                            int64_t stride_c, void *stream);

/* Prepared groups: a fixed set of products launched many times. Creation
 * validates the members as moa_gemm_grouped does, allocates the workspaces
 * (member tables, conditioned records) owned by the group, uploads the member
 * list once and captures the whole grouped
 * launch sequence (conditioning + one persistent contraction for split-BF16
 * members and one per FP8 term count, single launches for ONF and FP32
 * matrix-core members) in a HIP graph. Each moa_group_launch replays it on
 * `stream` (asynchronously) with the operand pointers given at creation;
 * results are bitwise those of moa_gemm. Creation synchronizes with the
 * device; replays of one group must not overlap each other.
 * moa_group_destroy waits for the group's outstanding work and frees it. */
typedef struct moa_group moa_group;
moa_status moa_group_create(const moa_gemm_desc *descs, int64_t count, moa_group **out);
moa_status moa_group_launch(moa_group *group, void *stream);
moa_status moa_group_destroy(moa_group *group);

/* The plan moa_gemm would use for `desc` (no launch; pointers may be null).
 * Returns the same argument errors as moa_gemm. */
moa_status moa_plan_query(const moa_gemm_desc *desc, moa_plan_info *out);

/* Autotuner. The planner starts from the static rule (below) and picks a
 * kernel instantiation from shape alone; moa_autotune times every
 * instantiation of desc's path on the caller's buffers (C is overwritten;
 * `reps` >= 1 timed runs each, after one warm-up) on `stream`, waits for
 * them, and records the fastest for desc's shape class -- (dtype, path,
 * FP8 term count, ceil(log2 m), ceil(log2 n), ceil(log2 p)). moa_gemm,
 * moa_gemm_grouped's single launches and moa_plan_query then use the
 * recorded instantiation for every product of that class unless
 * MOA_FLAG_VARIANT forces one. `chosen` (may be null) receives the plan and
 * `best_ms` (may be null) the time per run of the winner. Errors: as
 * moa_gemm; MOA_ERR_INVALID for reps < 1. */
moa_status moa_autotune(const moa_gemm_desc *desc, int32_t reps, void *stream,
                        moa_plan_info *chosen, double *best_ms);
/* Writes the recorded classes to a text file (one class per line) /
 * merges a file written by moa_autotune_save / forgets every record. */
moa_status moa_autotune_save(const char *path);
moa_status moa_autotune_load(const char *path);
moa_status moa_autotune_clear(void);

/* Block-size rule of section "Technical Details": the largest power of two b
 * with nblocks * b * elem_bytes <= budget_bytes (one block each of A, B and C
 * per processor memory: nblocks = 3). Returns 0 if none fits or an argument
 * is not positive. Pure host function. */
int64_t moa_static_block_components(int64_t budget_bytes, int64_t elem_bytes,
                                    int64_t nblocks);

/* Operand conditioning of the split-BF16 path, exposed so that it can be
 * checked on its own: X is rows x cols FP32 row-major (device);
 * hi[t] = RNE_bf16(X[t]), lo[t] = RNE_bf16(X[t] - hi[t]) as raw BF16 bit
 * patterns (uint16), written row-major with the same shape. Asynchronous.
 * Errors: MOA_ERR_INVALID for null pointers with rows*cols > 0. */
moa_status moa_split_bf16(const float *X, int64_t rows, int64_t cols,
                          uint16_t *hi, uint16_t *lo, void *stream);

/* Operand conditioning of the FP8 path, exposed for checking: for A (m x n)
 * writes e[i] (int32, per row) and qA (m x n E4M3 codes, row-major); for B
 * (n x p) writes f[j] (per column) and qB (n x p codes, row-major). With
 * two_term != 0 also writes the residual codes lA, lB (else they may be
 * null). Device pointers; asynchronous. */
moa_status moa_quantise_fp8(const float *A, int64_t m, int64_t n,
                            const float *B, int64_t p, int32_t two_term,
                            int32_t *e, uint8_t *qA, uint8_t *lA,
                            int32_t *f, uint8_t *qB, uint8_t *lB,
                            void *stream);

/* Error norm in FP64 on the device: out[0] = sum_t (X[t] - R[t])^2 and
 * out[1] = sum_t R[t]^2 over `count` elements, X of type `x_dtype`
 * (moa_dtype), R double. `out` is a device array of 2 doubles. The
 * normwise relative error is sqrt(out[0] / out[1]). Deterministic order.
 * Asynchronous. */
moa_status moa_error_norm(int64_t count, int32_t x_dtype, const void *X,
                          const double *R, double *out, void *stream);

/* Host-side check of the direct-to-LDS loads that the record-ring kernel of
 * `desc`'s plan would issue (split-BF16, scaled FP8 and the FP32 matrix-core
 * record variants; section "Dimension Lifting to Machine Coordinates": the
 * blocks of the lift may overhang the matrix). Walks every block, wave and
 * load of the launch on the host and counts loads that would read outside
 * their record array or buffer range, or whose offsets overflow 32 bits.
 * No device work; pointers in `desc` may be null. `loads` (may be null)
 * receives the number of loads per slab checked, `violations` the count found
 * (0 when every load is in bounds). Errors: as moa_plan_query;
 * MOA_ERR_UNSUPPORTED when the plan runs no record ring (ONF, the
 * register-staged FP32 variant). */
moa_status moa_diag_ring_loads(const moa_gemm_desc *desc, int64_t *loads, int64_t *violations);

/* ------------------------------------------------------------------------
 * Kernel timing (profiling aid). While enabled, every kernel the library
 * launches is bracketed by two HIP events recorded on the launch's own
 * stream; moa_trace_read folds the finished pairs into per-kernel totals.
 * ---------------------------------------------------------------------- */
typedef enum moa_kernel {
    MOA_K_ONF_F64 = 1,        /* plain ONF contraction, FP64 */
    MOA_K_ONF_F32 = 2,        /* plain ONF contraction, FP32 */
    MOA_K_MFMA_F32 = 3,       /* FP32 matrix-core product (record copies included) */
    MOA_K_SPLIT_BF16 = 4,     /* split-BF16 contraction (single product) */
    MOA_K_FP8 = 5,            /* scaled-FP8 contraction, one term */
    MOA_K_FP8_2TERM = 6,      /* scaled-FP8 contraction, two terms */
    MOA_K_SPLIT_PACK = 7,     /* split-BF16 operand conditioning */
    MOA_K_FP8_QUANT = 8,      /* FP8 operand conditioning */
    MOA_K_SPLIT_GROUPED = 9,  /* grouped persistent split-BF16 contraction */
    MOA_K_FP8_GROUPED = 10,   /* grouped persistent scaled-FP8 contraction */
    MOA_K_HADAMARD = 11,      /* Hadamard product */
    MOA_K_KRONECKER = 12,     /* Kronecker product */
    MOA_K_COUNT = 13
} moa_kernel;

typedef struct moa_trace_stat {
    int32_t kernel;           /* moa_kernel */
    int32_t reserved;
    int64_t launches;         /* completed launches folded in */
    double total_ms;          /* sum of their event-measured durations */
} moa_trace_stat;

/* Turns tracing on (non-zero) or off. Off by default. Thread-safe. */
moa_status moa_trace_enable(int32_t on);

/* Folds every finished event pair into the totals and writes one entry per
 * kernel kind with launches > 0 (at most `capacity`) to `out`, the number
 * written to `*count`. Pairs whose work has not finished are kept for the
 * next call (synchronize the streams first for complete totals). With
 * reset != 0 the totals are cleared after reading. Host memory only. */
moa_status moa_trace_read(moa_trace_stat *out, int32_t capacity, int32_t *count,
                          int32_t reset);

/* ------------------------------------------------------------------------
 * Serving: a request loop that admits products of mixed shapes under an HBM
 * budget and batches them into grouped launches on several streams
 * (continuous batching: requests that arrive while others run are admitted
 * as slots and memory free up). Not a construct of the paper; every request
 * computes Eq. 3 as moa_gemm does, bitwise the same result.
 *
 * Two kinds of request:
 *  - caller-owned: a moa_gemm_desc whose A, B, C are the caller's device
 *    memory (moa_serve_submit);
 *  - synthetic: (m, n, p, path, flags, seed) only (moa_serve_submit_synthetic).
 *    The server takes A, B and C from its own pool at admission and draws A
 *    and B on the device with moa_fill_synthetic's generator (A: operand 0,
 *    B: operand 1, both with the request's seed) right before the group's
 *    launch; C stays in the pool until the ticket is released.
 *
 * Memory: all device memory the server allocates -- synthetic operands and
 * results, and the scratch of every grouped launch, caller-owned requests
 * included -- comes from a pool whose total never exceeds hbm_budget_bytes.
 * A request counts against the budget from admission to completion with its
 * operands and result (caller-owned ones too) and the scratch it would take
 * alone; a synthetic request's C stays counted until it is released.
 *
 * Ordering: the server's streams do not wait for any stream of the caller.
 * The operands of a caller-owned request must be complete when it is
 * submitted (e.g. the stream that produced them synchronized), and requests
 * are unordered with respect to each other: two requests must not write the
 * same C, and one must not read a C another writes.
 * ---------------------------------------------------------------------- */
typedef struct moa_server moa_server;

typedef struct moa_serve_cfg {
    int64_t hbm_budget_bytes; /* bound on the bytes admitted requests hold
                                 (operands, result, scratch) and on the
                                 server's device memory */
    int32_t slots;            /* concurrent groups in flight (streams), >= 1 */
    int32_t max_group;        /* most requests per grouped launch, >= 1 */
    int32_t device;           /* HIP device ordinal */
    int32_t batch_window_us;  /* batching window, >= 0: a group is launched
                                 once it has max_group requests or its oldest
                                 request has waited this long (0: at once) */
    int64_t pool_reserve_bytes; /* device memory the pool takes at creation
                                 (0 .. budget); the pool grows beyond it on
                                 demand. Allocating while groups run can stall
                                 the device, so a serving loop reserves what
                                 its load will hold. */
} moa_serve_cfg;

/* A synthetic request: C (m x p, FP32, row-major) := A.B on `path` with
 * `flags` (as in moa_gemm_desc; no layout flags), A (m x n) and B (n x p)
 * drawn on the device from `seed`. */
typedef struct moa_synth_request {
    int64_t m, n, p;
    int32_t path;             /* moa_path */
    uint32_t flags;
    uint64_t seed;
} moa_synth_request;

typedef struct moa_req_info {
    int64_t t_submit_ns;      /* CLOCK_MONOTONIC at submit */
    int64_t t_admit_ns;       /* admitted under the budget */
    int64_t t_start_ns;       /* its group's launch was enqueued */
    int64_t t_done_ns;        /* completion observed by the scheduler */
    int32_t status;           /* moa_status of the request */
    int32_t group_size;       /* members of the launch it ran in */
} moa_req_info;

typedef struct moa_serve_state {
    int64_t held_bytes;       /* bytes counted against the budget now */
    int64_t peak_held_bytes;  /* largest held_bytes so far */
    int64_t pool_bytes;       /* device memory the server holds now */
    int64_t peak_pool_bytes;  /* largest pool_bytes so far */
    int64_t admitted, completed, failed, waiting;   /* request counts */
} moa_serve_state;

/* Reserves the pool and starts the scheduler thread. Errors:
 * MOA_ERR_INVALID (null, slots < 1, max_group < 1, budget <= 0, negative
 * window, a reserve outside 0 .. budget, no such device), MOA_ERR_NOMEM (the
 * reserve cannot be allocated), MOA_ERR_DEVICE. */
moa_status moa_serve_create(const moa_serve_cfg *cfg, moa_server **out);

/* Queues one caller-owned product (descriptor copied; see Ordering above).
 * Returns a ticket. Errors: argument errors as moa_gemm; MOA_ERR_NOMEM if
 * the request alone exceeds the whole budget. Thread-safe. */
moa_status moa_serve_submit(moa_server *srv, const moa_gemm_desc *desc,
                            uint64_t *ticket);

/* Queues one synthetic product. Errors: argument errors as moa_gemm for the
 * equivalent FP32 descriptor; MOA_ERR_INVALID for layout flags;
 * MOA_ERR_NOMEM if it alone exceeds the whole budget. A request that the
 * device cannot hold even with nothing else in the pool completes with
 * status MOA_ERR_NOMEM. Thread-safe. */
moa_status moa_serve_submit_synthetic(moa_server *srv, const moa_synth_request *req,
                                      uint64_t *ticket);

/* MOA_OK and the timestamps once the request is done (its C is final),
 * MOA_NOT_READY before, MOA_ERR_INVALID for an unknown ticket. A completed
 * ticket may be polled any number of times until it is released.
 * Thread-safe. */
moa_status moa_serve_poll(moa_server *srv, uint64_t ticket,
                          moa_req_info *out);

/* Device address of the C of a done request (the server's for a synthetic
 * one, valid until release; the caller's otherwise). MOA_NOT_READY before
 * completion, MOA_ERR_INVALID for an unknown ticket. */
moa_status moa_serve_result(moa_server *srv, uint64_t ticket, const void **C);

/* Synchronous copy of a done request's C (m p elements) to `dst` (host or
 * device memory of at least dst_bytes bytes). Errors as moa_serve_result;
 * MOA_ERR_INVALID if dst_bytes is too small; MOA_ERR_DEVICE for a failed
 * copy. */
moa_status moa_serve_read(moa_server *srv, uint64_t ticket, void *dst, int64_t dst_bytes);

/* Frees the record of a completed ticket (and a synthetic request's C);
 * later calls with it return MOA_ERR_INVALID. MOA_NOT_READY (nothing
 * changes) while the request runs, MOA_ERR_INVALID for an unknown or already
 * released ticket. Records and synthetic results of tickets never released
 * are kept until moa_serve_destroy and keep counting against the budget, so
 * a long-running server must release each ticket once it has read it.
 * Thread-safe. */
moa_status moa_serve_release(moa_server *srv, uint64_t ticket);

/* Waits until every submitted request is done. */
moa_status moa_serve_drain(moa_server *srv);

/* Budget and pool figures of the server (host call, thread-safe). */
moa_status moa_serve_stats(moa_server *srv, moa_serve_state *out);

/* Drains, stops the scheduler and frees the server with its pool. */
moa_status moa_serve_destroy(moa_server *srv);

/* Synthetic operand draw on the device, asynchronous on `stream`: X[e] for
 * e < count (FP32, 4-byte aligned device memory) gets element e of operand
 * `operand` for `seed`. Generator: Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, SC 2011); pair q = e / 2 draws the block with counter
 * (q mod 2^32, q / 2^32, operand, 0) and key (seed mod 2^32, seed / 2^32);
 * element 2q takes words 0 and 1, element 2q + 1 words 2 and 3; with S the
 * sum of the four 16-bit halves of its two words, the value is the FP32
 * product (2 S - 262140) * c, c the FP32 value nearest sqrt(3) * 2^-17 (a
 * centred sum of four uniform variates: mean 0, variance 1). Errors:
 * MOA_ERR_SHAPE (count < 0), MOA_ERR_INVALID (null or misaligned X),
 * MOA_ERR_DEVICE. */
moa_status moa_fill_synthetic(float *X, int64_t count, uint64_t seed, uint32_t operand,
                              void *stream);

/* Static string for a status code. */
const char *moa_status_string(moa_status s);

/* Thread-local description of the last error returned on this thread
 * ("" if none). Valid until the next call on the same thread. */
const char *moa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MOA_H */
