// Internal declarations shared by the HIP kernels and the C-ABI runtime.
// Nothing here is part of the public ABI (include/moa.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "moa.h"

namespace moa {

// ---------------------------------------------------------------- errors --
void set_last_error(const std::string &msg);
moa_status fail(moa_status s, const char *fmt, ...)
    __attribute__((format(printf, 2, 3)));
moa_status hip_fail(hipError_t e, const char *what);

// ----------------------------------------------------------------- plans --
// Kernel identities (reported through moa_plan_info::kernel).
enum KernelId : int32_t {
    K_NONE = 0,
    K_ONF_F64 = 1,
    K_ONF_F32 = 2,
    K_MFMA_F32 = 3,
    K_SPLIT_BF16 = 4,
    K_FP8 = 5,
    K_FP8_2TERM = 6,
};

// The dimension lift of one product: i -> (workgroup row block, lane rows),
// j -> (workgroup column block, lane columns), k -> (LDS slab, in-slab).
struct Plan {
    moa_path path = MOA_PATH_AUTO;
    KernelId kernel = K_NONE;
    int variant = 0;          // index into the kernel's instantiation table
    int tile_m = 0, tile_n = 0, tile_k = 0;
    int wave_m = 0, wave_n = 0;
    int lane_m = 0, lane_n = 0;
    int threads = 256;
    int lds_bytes = 0;
    int64_t workgroups = 0;
    int64_t workspace_bytes = 0;
    int64_t static_components = 0;
    bool tuned = false;
    int split_k = 1;          // k chunks summed by separate workgroups (ring paths)
    int64_t partial_offset = 0;   // byte offset of the split-k partials in the workspace
};

// A descriptor with a column-major C rewritten as the product C^T = B^T A^T
// with a row-major result: A and B swap (with their layouts flipped: a
// row-major A read as A^T is column-major), m and p swap. Other descriptors
// are returned unchanged. The rewritten descriptor has no MOA_FLAG_C_COL.
inline moa_gemm_desc row_major_result(const moa_gemm_desc &d) {
    if (!(d.flags & MOA_FLAG_C_COL)) return d;
    moa_gemm_desc t = d;
    t.m = d.p;
    t.p = d.m;
    t.A = d.B;
    t.B = d.A;
    uint32_t f = d.flags & ~MOA_FLAG_LAYOUT_MASK;
    if (!(d.flags & MOA_FLAG_B_COL)) f |= MOA_FLAG_A_COL;
    if (!(d.flags & MOA_FLAG_A_COL)) f |= MOA_FLAG_B_COL;
    t.flags = f;
    return t;
}
inline bool has_col_operand(const moa_gemm_desc &d) { return (d.flags & MOA_FLAG_LAYOUT_MASK) != 0; }

// Term count of a scaled-FP8 descriptor: two unless MOA_FLAG_FP8_ONE_TERM.
inline bool fp8_two_term(const moa_gemm_desc &d) { return !(d.flags & MOA_FLAG_FP8_ONE_TERM); }

// Chunk count asked for by MOA_FLAG_SPLIT_K (0: the planner decides, 1: none).
inline int split_k_requested(const moa_gemm_desc &d) { return (int)((d.flags & MOA_FLAG_SPLIT_K_MASK) >> 16); }
// Chunks actually used for S slabs: ceil(S / ceil(S / c)), so none is empty.
inline int split_k_chunks(int requested, int64_t S) {
    if (requested <= 1 || S <= 1) return 1;
    const int64_t per = (S + requested - 1) / requested;
    return (int)((S + per - 1) / per);
}

// Validates `d` (shapes, pointers, enums, aliasing) without touching the
// device. `need_ptrs` = false skips pointer checks (plan queries).
moa_status validate(const moa_gemm_desc &d, bool need_ptrs);
moa_path resolve_path(const moa_gemm_desc &d);
moa_status make_plan(const moa_gemm_desc &d, Plan *out);
// Whether the plan of `d` sums k in chunks over separate workgroups (asked
// for or chosen by the planner).
inline bool plans_split_k(const moa_gemm_desc &d) {
    Plan pl;
    return d.m > 0 && d.p > 0 && make_plan(d, &pl) == MOA_OK && pl.split_k > 1;
}

// gfx950 constants used by the static rule and the planner.
constexpr int64_t kL1Bytes = 32 * 1024;        // vector L1 per CU
constexpr int64_t kLdsBytes = 160 * 1024;      // LDS per CU
constexpr int kNumCUs = 256;
constexpr int kNumXCDs = 8;

int64_t static_block_components(int64_t budget, int64_t elem, int64_t nblocks);

// Autotuner table: shape class -> variant (-1 if none recorded).
int tuned_variant(const moa_gemm_desc &d, moa_path path);
void record_tuned_variant(const moa_gemm_desc &d, moa_path path, int variant, double ms);
int variant_count(const moa_gemm_desc &d, moa_path path);
moa_status autotune_save(const char *path);
moa_status autotune_load(const char *path);
void autotune_clear();

// ----------------------------------------------------------------- trace --
// Brackets the launches made in its lifetime with events on `stream` while
// tracing is enabled (moa_trace_enable); a no-op otherwise.
class TraceScope {
  public:
    TraceScope(int32_t kernel, hipStream_t stream);
    ~TraceScope();
    TraceScope(const TraceScope &) = delete;
    TraceScope &operator=(const TraceScope &) = delete;

  private:
    int32_t kernel_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr;
};

// --------------------------------------------------------------- kernels --
// Each launcher enqueues the whole product for `d` on `stream` using `plan`
// and returns the first HIP error.
hipError_t launch_onf(const moa_gemm_desc &d, const Plan &plan, hipStream_t stream);
int onf_variant_count(moa_dtype t);
void onf_variant_shape(moa_dtype t, int v, Plan *p);
int onf_ring_variant(moa_dtype t);           // the direct-load ring kernel (row-major operands)
bool onf_ring_fits(moa_dtype t, int64_t n, int64_t p);

// FP32 matrix cores: variants 0, 1 run the record ring (workspace for the
// records), mfma_f32_staged_variant() the register-staged kernel (none).
hipError_t launch_mfma_f32(const moa_gemm_desc &d, const Plan &plan, void *workspace, hipStream_t stream);
void mfma_f32_shape(int variant, Plan *p);
int mfma_f32_variant_count();
int mfma_f32_staged_variant();
int mfma_f32_default_variant(int64_t m, int64_t p);
int64_t mfma_f32_workspace_bytes(int64_t m, int64_t n, int64_t p, int variant);

hipError_t launch_split_bf16(const moa_gemm_desc &d, const Plan &plan, void *workspace,
                             hipStream_t stream);
hipError_t launch_split_pack(const moa_gemm_desc &d, void *workspace, hipStream_t stream);
void split_bf16_shape(int variant, Plan *p);
int split_bf16_variant_count();
int split_bf16_default_variant(int64_t m, int64_t p);   // the planner's default block
int64_t split_bf16_workspace_bytes(int64_t m, int64_t n, int64_t p);
// Grouped split-BF16: all `members` in one conditioning pass and one
// persistent launch. `host_staging` is pinned memory of at least
// split_grouped_desc_bytes(count) bytes that stays untouched until the
// stream has passed this call.
int64_t split_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count);
// Whether a split-BF16 member fits the persistent launch's 32-bit offsets
// (else it runs as a single launch).
bool split_grouped_fits(const moa_gemm_desc &d);
int64_t split_grouped_desc_bytes(const moa_gemm_desc *const *members, int count);
// `host_staging_dev`: the staging buffer's address in the device's address
// space (null: the table goes up by a copy instead of being read in place).
hipError_t launch_split_grouped(const moa_gemm_desc *const *members, int count, int variant, void *workspace,
                                void *host_staging, const void *host_staging_dev, hipStream_t stream);
// Persistent split-BF16 kernels of a grouped launch (blocks 128 x 128 split
// once with three or two blocks per CU, 128 x 128 split in registers,
// 64 x 128, 128 x 64), the static rule's choice among them, and the choice a
// grouped launch makes: `forced` when >= 0, else the autotuner's record for
// the members' class, else the static rule.
int split_grouped_variant_count();
int split_grouped_default_variant(const moa_gemm_desc *const *members, int count);
int split_grouped_choose(const moa_gemm_desc *const *members, int count, int forced, bool *tuned);
int tuned_group_variant(const moa_gemm_desc *const *members, int count);
void record_tuned_group_variant(const moa_gemm_desc *const *members, int count, int variant, double ms);
// The two halves of launch_split_grouped: host layout (returns the sizes of
// the contraction and conditioning work lists; the member array to upload is
// in host_staging) and the device sequence, which allocates, copies and clears
// nothing (graph-capturable).
struct GroupedWork {
    int64_t tiles;                      // contraction tiles over all members
    int64_t pack_items;                 // conditioning items over all members
    int variant;                        // persistent kernel
    int64_t table_used;                 // bytes of the member table the launch reads (a prefix)
};
GroupedWork split_grouped_layout(const moa_gemm_desc *const *members, int count, void *workspace,
                                 void *host_staging, int variant);
hipError_t split_grouped_enqueue(void *workspace, int count, const GroupedWork &work, hipStream_t stream);

hipError_t launch_fp8(const moa_gemm_desc &d, const Plan &plan, void *workspace,
                      hipStream_t stream);
void fp8_shape(bool two_term, int variant, Plan *p);
int fp8_variant_count(bool two_term);
int64_t fp8_workspace_bytes(int64_t m, int64_t n, int64_t p, bool two_term);

// Grouped FP8 (members of one term count, validated by the caller): one
// conditioning pass over all members and one persistent contraction. The
// layout/enqueue split mirrors the split-BF16 one (graph-capturable enqueue).
struct Fp8GroupWork {
    int64_t tiles;                      // contraction tiles over all members
    int64_t scale_items;                // exponent / amax items
    int64_t pack_items;                 // record items
    int64_t clear_words;                // 32-bit words cleared first (counter + column amax)
    int64_t table_offset;               // byte offset of the member table in the workspace
};
int64_t fp8_grouped_workspace_bytes(const moa_gemm_desc *const *members, int count, bool two_term);
int64_t fp8_grouped_desc_bytes(int count);
Fp8GroupWork fp8_grouped_layout(const moa_gemm_desc *const *members, int count, bool two_term, void *workspace,
                                void *host_staging);
hipError_t fp8_grouped_enqueue(void *workspace, int count, bool two_term, const Fp8GroupWork &work,
                               hipStream_t stream);
hipError_t launch_fp8_grouped(const moa_gemm_desc *const *members, int count, bool two_term, void *workspace,
                              void *host_staging, const void *host_staging_dev, hipStream_t stream);

hipError_t launch_split_only(const float *X, int64_t count, uint16_t *hi, uint16_t *lo,
                             hipStream_t stream);
hipError_t launch_quantise_fp8(const float *A, int64_t m, int64_t n, const float *B,
                               int64_t p, bool two_term, int32_t *e, uint8_t *qA,
                               uint8_t *lA, int32_t *f, uint8_t *qB, uint8_t *lB,
                               uint32_t *amax_scratch, hipStream_t stream);
// Synthetic operand fill (Philox4x32-10 counter-based draws; synthetic.hip).
hipError_t launch_synthetic(float *X, int64_t count, uint64_t seed, uint32_t tag, hipStream_t stream);
hipError_t launch_error_norm(int64_t count, moa_dtype xt, const void *X, const double *R,
                             double *out, double *partials, int nblocks, hipStream_t stream);

// Runs one product: plan + scratch + launch. Used by moa_gemm and by the
// grouped and serving paths for members that run alone.
moa_status run_gemm(const moa_gemm_desc &d, hipStream_t stream);
// The same with the workspace given: `fixed_ws` of `fixed_bytes` bytes
// (MOA_ERR_NOMEM if the plan needs more), or the cached scratch when null.
moa_status run_gemm_in(const moa_gemm_desc &d, hipStream_t stream, void *fixed_ws, int64_t fixed_bytes);

// Grouped products (validated by the caller): split-BF16 members in one
// persistent launch sequence, scaled-FP8 members in one per term count, the
// others (and split-k or column-major members) one after another.
// A caller-owned block of device memory that a grouped launch carves its
// scratch from (256-byte aligned pieces, in launch order) instead of the
// scratch cache.
struct ScratchArena {
    void *base = nullptr;
    int64_t size = 0;
    int64_t used = 0;
};
// `split_k` (optional): per member, whether its plan splits k (as the caller
// already planned it), so that members are not planned twice.
moa_status run_grouped(const moa_gemm_desc *descs, int64_t count, hipStream_t stream,
                       ScratchArena *arena = nullptr, int split_variant = -1, const char *split_k = nullptr);
// Bytes of scratch run_grouped takes from an arena for these members.
int64_t grouped_scratch_bytes(const moa_gemm_desc *descs, int64_t count);
// Scratch bytes of one product under its plan (0 for empty products).
int64_t gemm_workspace_bytes(const moa_gemm_desc &d);
moa_status check_group_overlap(const moa_gemm_desc *descs, int64_t count);

// Scratch of one call on `stream` (scratch.cpp): cached device buffers,
// reused on the same stream at once and across streams once their last use
// has completed; the stream-ordered allocator during graph capture.
moa_status scratch_alloc(void **ptr, int64_t bytes, hipStream_t stream);
void scratch_free(void *ptr, hipStream_t stream);

}  // namespace moa
