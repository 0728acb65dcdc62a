// C-ABI entry points: argument checks (Eq. 1-2 shapes and index bounds),
// planning, scratch and kernel dispatch. No exception crosses the ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "moa_internal.h"
#include "ring_gemm.h"

namespace moa {

namespace {
thread_local std::string t_last_error;
}  // namespace

void set_last_error(const std::string &msg) { t_last_error = msg; }

moa_status fail(moa_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return s;
}

moa_status hip_fail(hipError_t e, const char *what) {
    return fail(MOA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static bool mul_ok(int64_t a, int64_t b, int64_t *out) {
    if (a == 0 || b == 0) { *out = 0; return true; }
    if (a > INT64_MAX / b) return false;
    *out = a * b;
    return true;
}

moa_status validate(const moa_gemm_desc &d, bool need_ptrs) {
    if (d.m < 0 || d.n < 0 || d.p < 0)
        return fail(MOA_ERR_SHAPE, "negative shape <%lld, %lld, %lld>", (long long)d.m,
                    (long long)d.n, (long long)d.p);
    if (d.dtype != MOA_F64 && d.dtype != MOA_F32) return fail(MOA_ERR_INVALID, "unknown dtype %d", d.dtype);
    if (d.path < MOA_PATH_AUTO || d.path > MOA_PATH_FP8_SCALED)
        return fail(MOA_ERR_INVALID, "unknown path %d", d.path);
    if (d.flags & ~(MOA_FLAG_FP8_TWO_TERM | MOA_FLAG_FP8_ONE_TERM | MOA_FLAG_VARIANT_MASK | MOA_FLAG_SPLIT_K_MASK |
                    MOA_FLAG_LAYOUT_MASK))
        return fail(MOA_ERR_INVALID, "unknown flag bits 0x%x", d.flags);
    if ((d.flags & MOA_FLAG_FP8_TWO_TERM) && (d.flags & MOA_FLAG_FP8_ONE_TERM))
        return fail(MOA_ERR_INVALID, "MOA_FLAG_FP8_ONE_TERM and MOA_FLAG_FP8_TWO_TERM both set");
    const moa_path path = resolve_path(d);
    if (d.dtype == MOA_F64 && path != MOA_PATH_ONF)
        return fail(MOA_ERR_UNSUPPORTED, "FP64 runs on the ONF path only (path %d)", (int)path);
    if (split_k_requested(d) > 1 && path != MOA_PATH_SPLIT_BF16 && path != MOA_PATH_FP8_SCALED)
        return fail(MOA_ERR_UNSUPPORTED, "split-k needs the split-BF16 or FP8 path (path %d)", (int)path);
    const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
    int64_t na, nb, nc, ba, bb, bc;
    if (!mul_ok(d.m, d.n, &na) || !mul_ok(d.n, d.p, &nb) || !mul_ok(d.m, d.p, &nc) ||
        !mul_ok(na, es, &ba) || !mul_ok(nb, es, &bb) || !mul_ok(nc, es, &bc))
        return fail(MOA_ERR_SHAPE, "element count overflow");
    if (!need_ptrs) return MOA_OK;
    if ((na > 0 && !d.A) || (nb > 0 && !d.B) || (nc > 0 && !d.C))
        return fail(MOA_ERR_INVALID, "null matrix pointer for a non-empty operand");
    if (nc > 0) {
        const uintptr_t c0 = (uintptr_t)d.C, c1 = c0 + (uintptr_t)bc;
        auto overlaps = [&](const void *x, int64_t bytes) {
            if (bytes == 0) return false;
            const uintptr_t x0 = (uintptr_t)x, x1 = x0 + (uintptr_t)bytes;
            return x0 < c1 && c0 < x1;
        };
        if (overlaps(d.A, ba) || overlaps(d.B, bb))
            return fail(MOA_ERR_INVALID, "C overlaps A or B");
    }
    const uintptr_t align = (uintptr_t)es;
    if (((uintptr_t)d.A % align) || ((uintptr_t)d.B % align) || ((uintptr_t)d.C % align))
        return fail(MOA_ERR_INVALID, "matrix pointers must be aligned to the element size");
    return MOA_OK;
}

moa_status run_gemm_in(const moa_gemm_desc &d_in, hipStream_t stream, void *fixed_ws, int64_t fixed_bytes) {
    if (d_in.m == 0 || d_in.p == 0) return MOA_OK;
    const moa_gemm_desc d = row_major_result(d_in);
    Plan pl;
    moa_status s = make_plan(d, &pl);
    if (s != MOA_OK) return s;
    if (fixed_ws && pl.workspace_bytes > fixed_bytes)
        return fail(MOA_ERR_NOMEM, "the product needs %lld bytes of scratch, the fixed scratch array holds %lld",
                    (long long)pl.workspace_bytes, (long long)fixed_bytes);
    void *ws = fixed_ws;
    const bool cached = !fixed_ws && pl.path != MOA_PATH_ONF;
    if (cached && (s = scratch_alloc(&ws, pl.workspace_bytes, stream)) != MOA_OK) return s;
    hipError_t e = hipSuccess;
    switch (pl.path) {
    case MOA_PATH_ONF: {
        TraceScope ts(pl.kernel, stream);
        e = launch_onf(d, pl, stream);
        break;
    }
    case MOA_PATH_MFMA_F32: {
        TraceScope ts(pl.kernel, stream);      // record copies and contraction
        e = launch_mfma_f32(d, pl, ws, stream);
        break;
    }
    case MOA_PATH_SPLIT_BF16: e = launch_split_bf16(d, pl, ws, stream); break;
    case MOA_PATH_FP8_SCALED: e = launch_fp8(d, pl, ws, stream); break;
    default: s = fail(MOA_ERR_INVALID, "unresolved path");
    }
    if (cached) scratch_free(ws, stream);
    if (s != MOA_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return MOA_OK;
}

moa_status run_gemm(const moa_gemm_desc &d, hipStream_t stream) { return run_gemm_in(d, stream, nullptr, 0); }

int64_t gemm_workspace_bytes(const moa_gemm_desc &d) {
    if (d.m == 0 || d.p == 0) return 0;
    Plan pl;
    if (make_plan(row_major_result(d), &pl) != MOA_OK) return 0;
    return pl.workspace_bytes;
}

}  // namespace moa

using namespace moa;

extern "C" {

moa_status moa_gemm(const moa_gemm_desc *desc, void *stream) {
    try {
        if (!desc) return fail(MOA_ERR_INVALID, "null descriptor");
        moa_status s = validate(*desc, true);
        if (s != MOA_OK) return s;
        return run_gemm(*desc, static_cast<hipStream_t>(stream));
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_plan_query(const moa_gemm_desc *desc, moa_plan_info *out) {
    try {
        if (!desc || !out) return fail(MOA_ERR_INVALID, "null argument");
        moa_status s = validate(*desc, false);
        if (s != MOA_OK) return s;
        Plan pl;
        s = make_plan(*desc, &pl);
        if (s != MOA_OK) return s;
        std::memset(out, 0, sizeof *out);
        out->path = pl.path;
        out->kernel = pl.kernel;
        out->tile_m = pl.tile_m;
        out->tile_n = pl.tile_n;
        out->tile_k = pl.tile_k;
        out->wave_m = pl.wave_m;
        out->wave_n = pl.wave_n;
        out->lane_m = pl.lane_m;
        out->lane_n = pl.lane_n;
        out->threads = pl.threads;
        out->lds_bytes = pl.lds_bytes;
        out->workgroups = pl.workgroups;
        out->workspace_bytes = pl.workspace_bytes;
        out->static_components = pl.static_components;
        out->variant = pl.variant;
        out->tuned = pl.tuned ? 1 : 0;
        out->split_k = pl.split_k;
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_autotune(const moa_gemm_desc *desc, int32_t reps, void *stream, moa_plan_info *chosen,
                        double *best_ms) {
    try {
        if (!desc) return fail(MOA_ERR_INVALID, "null descriptor");
        if (reps < 1) return fail(MOA_ERR_INVALID, "reps must be >= 1");
        moa_status s = validate(*desc, true);
        if (s != MOA_OK) return s;
        hipStream_t st = static_cast<hipStream_t>(stream);
        const moa_path path = resolve_path(*desc);
        if (desc->m > 0 && desc->p > 0) {
            const int nv = variant_count(*desc, path);
            hipEvent_t a = nullptr, b = nullptr;
            hipError_t e = hipEventCreate(&a);
            if (e == hipSuccess) e = hipEventCreate(&b);
            if (e != hipSuccess) {
                if (a) (void)hipEventDestroy(a);
                return hip_fail(e, "hipEventCreate");
            }
            int best = -1;
            float best_t = 0.0f;
            for (int v = 0; v < nv && s == MOA_OK; ++v) {
                moa_gemm_desc d = *desc;
                d.path = path;
                d.flags = (d.flags & ~MOA_FLAG_VARIANT_MASK) | MOA_FLAG_VARIANT(v);
                Plan pl;
                if (make_plan(d, &pl) != MOA_OK) continue;       // e.g. a grid limit
                if ((s = run_gemm(d, st)) != MOA_OK) break;      // warm-up
                (void)hipEventRecord(a, st);
                for (int r = 0; r < reps && s == MOA_OK; ++r) s = run_gemm(d, st);
                (void)hipEventRecord(b, st);
                if ((e = hipEventSynchronize(b)) != hipSuccess) {
                    s = hip_fail(e, "autotune timing");
                    break;
                }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, a, b);
                ms /= (float)reps;
                if (best < 0 || ms < best_t) {
                    best = v;
                    best_t = ms;
                }
            }
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (s != MOA_OK) return s;
            if (best < 0) return fail(MOA_ERR_UNSUPPORTED, "no variant of path %d can run this shape", (int)path);
            record_tuned_variant(*desc, path, best, best_t);
            if (best_ms) *best_ms = best_t;
        }
        if (chosen) return moa_plan_query(desc, chosen);
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_autotune_save(const char *path) {
    if (!path) return fail(MOA_ERR_INVALID, "null path");
    return autotune_save(path);
}

moa_status moa_autotune_load(const char *path) {
    if (!path) return fail(MOA_ERR_INVALID, "null path");
    return autotune_load(path);
}

moa_status moa_autotune_clear(void) {
    autotune_clear();
    return MOA_OK;
}

int64_t moa_static_block_components(int64_t budget_bytes, int64_t elem_bytes, int64_t nblocks) {
    return static_block_components(budget_bytes, elem_bytes, nblocks);
}

moa_status moa_split_bf16(const float *X, int64_t rows, int64_t cols, uint16_t *hi, uint16_t *lo,
                          void *stream) {
    if (rows < 0 || cols < 0) return fail(MOA_ERR_SHAPE, "negative shape");
    int64_t count;
    if (!mul_ok(rows, cols, &count)) return fail(MOA_ERR_SHAPE, "element count overflow");
    if (count == 0) return MOA_OK;
    if (!X || !hi || !lo) return fail(MOA_ERR_INVALID, "null pointer");
    hipError_t e = launch_split_only(X, count, hi, lo, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "split launch");
    return MOA_OK;
}

moa_status moa_quantise_fp8(const float *A, int64_t m, int64_t n, const float *B, int64_t p,
                            int32_t two_term, int32_t *e, uint8_t *qA, uint8_t *lA, int32_t *f,
                            uint8_t *qB, uint8_t *lB, void *stream) {
    if (m < 0 || n < 0 || p < 0) return fail(MOA_ERR_SHAPE, "negative shape");
    int64_t na, nb;
    if (!mul_ok(m, n, &na) || !mul_ok(n, p, &nb)) return fail(MOA_ERR_SHAPE, "element count overflow");
    if ((na > 0 && (!A || !qA)) || (nb > 0 && (!B || !qB)) || (m > 0 && !e) || (p > 0 && !f))
        return fail(MOA_ERR_INVALID, "null pointer");
    if (two_term && ((na > 0 && !lA) || (nb > 0 && !lB)))
        return fail(MOA_ERR_INVALID, "two-term needs residual outputs");
    if (m + p == 0) return MOA_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *amax = nullptr;
    moa_status s = scratch_alloc(&amax, 4 * (m + p), st);
    if (s != MOA_OK) return s;
    hipError_t err = launch_quantise_fp8(A, m, n, B, p, two_term != 0, e, qA, lA, f, qB, lB,
                                         static_cast<uint32_t *>(amax), st);
    scratch_free(amax, st);
    if (err != hipSuccess) return hip_fail(err, "quantise launch");
    return MOA_OK;
}

moa_status moa_error_norm(int64_t count, int32_t x_dtype, const void *X, const double *R,
                          double *out, void *stream) {
    if (count < 0) return fail(MOA_ERR_SHAPE, "negative count");
    if (x_dtype != MOA_F64 && x_dtype != MOA_F32) return fail(MOA_ERR_INVALID, "unknown dtype");
    if (!out || (count > 0 && (!X || !R))) return fail(MOA_ERR_INVALID, "null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    constexpr int kBlocks = 1024;
    void *partials = nullptr;
    moa_status s = scratch_alloc(&partials, 2 * kBlocks * sizeof(double), st);
    if (s != MOA_OK) return s;
    hipError_t e = launch_error_norm(count, (moa_dtype)x_dtype, X, R, out,
                                     static_cast<double *>(partials), kBlocks, st);
    scratch_free(partials, st);
    if (e != hipSuccess) return hip_fail(e, "error-norm launch");
    return MOA_OK;
}

moa_status moa_diag_ring_loads(const moa_gemm_desc *desc, int64_t *loads, int64_t *violations) {
    try {
        if (!desc || !violations) return fail(MOA_ERR_INVALID, "null argument");
        moa_status s = validate(*desc, false);
        if (s != MOA_OK) return s;
        const moa_gemm_desc d = row_major_result(*desc);
        Plan pl;
        if ((s = make_plan(d, &pl)) != MOA_OK) return s;
        const bool ring = pl.path == MOA_PATH_SPLIT_BF16 || pl.path == MOA_PATH_FP8_SCALED ||
                          (pl.path == MOA_PATH_MFMA_F32 && pl.workspace_bytes > 0);
        if (!ring) return fail(MOA_ERR_UNSUPPORTED, "path %d runs no record ring", (int)pl.path);
        const int nrec = pl.path == MOA_PATH_FP8_SCALED && fp8_two_term(d) ? 2 : 1;
        const int64_t S = (d.n + pl.tile_k - 1) / pl.tile_k;
        if (d.m == 0 || d.p == 0 || S == 0) {
            if (loads) *loads = 0;
            *violations = 0;
            return MOA_OK;
        }
        *violations = ring::check_loads(pl.tile_m, pl.tile_n, pl.wave_m, pl.wave_n, nrec, d.m, d.p, S, loads);
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

const char *moa_status_string(moa_status s) {
    switch (s) {
    case MOA_OK: return "MOA_OK";
    case MOA_ERR_INVALID: return "MOA_ERR_INVALID";
    case MOA_ERR_SHAPE: return "MOA_ERR_SHAPE";
    case MOA_ERR_UNSUPPORTED: return "MOA_ERR_UNSUPPORTED";
    case MOA_ERR_NOMEM: return "MOA_ERR_NOMEM";
    case MOA_ERR_DEVICE: return "MOA_ERR_DEVICE";
    case MOA_NOT_READY: return "MOA_NOT_READY";
    }
    return "MOA_UNKNOWN_STATUS";
}

const char *moa_last_error(void) { return t_last_error.c_str(); }

}  // extern "C"
