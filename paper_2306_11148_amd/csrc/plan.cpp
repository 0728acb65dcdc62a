// Planner: the dimension lift of a product onto gfx950.
//
// Seed rule (section "Technical Details"): three blocks -- one each of A, B
// and C -- of b components of the element type are sized to one processor's
// memory; b is a power of two and only the component count matters, not the
// block's aspect ratio. On gfx950 the processor memory that plays the V100
// L1's role is the CU's 32 KB vector L1, which gives 1024 FP64 components
// (32 x 32, as on the V100) and 2048 FP32 components (32 x 64). That block is
// the first entry of each ONF instantiation table. Larger blocks, staged in
// the 160 KB LDS with the C block held in registers, are the neighbours the
// planner (and the autotuner) choose among: a launch must also cover the 256
// CUs several times over, so the planner takes the largest block that still
// yields at least one workgroup per CU and falls back to the smallest.
#include <array>
#include <vector>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include <algorithm>

#include "moa_internal.h"

namespace moa {

namespace {

using ClassKey = std::array<int, 6>;
struct Tuned { int variant; double ms; };
std::mutex g_tune_mu;
std::map<ClassKey, Tuned> g_tuned;

int ceil_log2(int64_t x) {
    int r = 0;
    while (r < 62 && (int64_t(1) << r) < x) ++r;
    return r;
}

ClassKey class_key(const moa_gemm_desc &d, moa_path path) {
    return {d.dtype, (int)path, path == MOA_PATH_FP8_SCALED && fp8_two_term(d) ? 2 : 1, ceil_log2(d.m),
            ceil_log2(d.n), ceil_log2(d.p)};
}

// Class of a grouped launch's persistent split-BF16 members: member count and
// the medians of m, n and p, each as ceil(log2); marked by a path code no
// single product has.
constexpr int kGroupClass = 16;
ClassKey group_key(const moa_gemm_desc *const *members, int count) {
    std::vector<int64_t> m(count), n(count), p(count);
    for (int k = 0; k < count; ++k) {
        m[k] = members[k]->m;
        n[k] = members[k]->n;
        p[k] = members[k]->p;
    }
    auto median = [](std::vector<int64_t> &v) {
        std::nth_element(v.begin(), v.begin() + (long)(v.size() / 2), v.end());
        return v[v.size() / 2];
    };
    return {MOA_F32, kGroupClass, ceil_log2(count), ceil_log2(median(m)), ceil_log2(median(n)), ceil_log2(median(p))};
}

}  // namespace

int tuned_group_variant(const moa_gemm_desc *const *members, int count) {
    if (count <= 0) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(group_key(members, count));
    return it == g_tuned.end() ? -1 : it->second.variant;
}

void record_tuned_group_variant(const moa_gemm_desc *const *members, int count, int variant, double ms) {
    if (count <= 0) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[group_key(members, count)] = {variant, ms};
}

int split_grouped_choose(const moa_gemm_desc *const *members, int count, int forced, bool *tuned) {
    if (tuned) *tuned = false;
    if (forced >= 0) return forced;
    const int t = tuned_group_variant(members, count);
    if (t >= 0) {
        if (tuned) *tuned = true;
        return t;
    }
    return split_grouped_default_variant(members, count);
}

int tuned_variant(const moa_gemm_desc &d, moa_path path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(class_key(d, path));
    return it == g_tuned.end() ? -1 : it->second.variant;
}

void record_tuned_variant(const moa_gemm_desc &d, moa_path path, int variant, double ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[class_key(d, path)] = {variant, ms};
}

int variant_count(const moa_gemm_desc &d, moa_path path) {
    switch (path) {
    case MOA_PATH_ONF: return onf_variant_count((moa_dtype)d.dtype);
    case MOA_PATH_SPLIT_BF16: return split_bf16_variant_count();
    case MOA_PATH_MFMA_F32: return mfma_f32_variant_count();
    case MOA_PATH_FP8_SCALED: return fp8_variant_count(fp8_two_term(d));
    default: return 1;
    }
}

moa_status autotune_save(const char *path) {
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(MOA_ERR_INVALID, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::fprintf(f, "# moa autotune v1: dtype path terms log2m log2n log2p variant ms "
                    "(path %d: grouped split-BF16, fields count and median m, n, p)\n", kGroupClass);
    for (const auto &kv : g_tuned)
        std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", kv.first[0], kv.first[1], kv.first[2], kv.first[3],
                     kv.first[4], kv.first[5], kv.second.variant, kv.second.ms);
    std::fclose(f);
    return MOA_OK;
}

moa_status autotune_load(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(MOA_ERR_INVALID, "cannot read %s", path);
    char line[256];
    std::map<ClassKey, Tuned> add;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        ClassKey k;
        Tuned t;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %lf", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &t.variant,
                        &t.ms) != 8) {
            std::fclose(f);
            return fail(MOA_ERR_INVALID, "malformed line in %s: %s", path, line);
        }
        moa_gemm_desc probe{};
        probe.dtype = k[0];
        probe.flags = k[2] == 2 ? 0 : MOA_FLAG_FP8_ONE_TERM;
        const bool group = k[1] == kGroupClass && k[0] == MOA_F32;
        const int nvar = group ? split_grouped_variant_count()
                               : (k[1] < MOA_PATH_ONF || k[1] > MOA_PATH_FP8_SCALED) ? 0
                                                                                      : variant_count(probe, (moa_path)k[1]);
        if ((!group && (k[1] < MOA_PATH_ONF || k[1] > MOA_PATH_FP8_SCALED)) || (k[0] != MOA_F64 && k[0] != MOA_F32) ||
            t.variant < 0 || t.variant >= nvar) {
            std::fclose(f);
            return fail(MOA_ERR_INVALID, "out-of-range entry in %s: %s", path, line);
        }
        add[k] = t;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : add) g_tuned[kv.first] = kv.second;
    return MOA_OK;
}

void autotune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

int64_t static_block_components(int64_t budget, int64_t elem, int64_t nblocks) {
    if (budget <= 0 || elem <= 0 || nblocks <= 0) return 0;
    if (nblocks > budget / elem) return 0;
    int64_t b = 1;
    // double while nblocks * 2b * elem <= budget (no overflow: b <= budget)
    while (2 * b <= budget / (nblocks * elem)) b *= 2;
    return b;
}

moa_path resolve_path(const moa_gemm_desc &d) {
    if (d.path != MOA_PATH_AUTO) return (moa_path)d.path;
    return d.dtype == MOA_F64 ? MOA_PATH_ONF : MOA_PATH_SPLIT_BF16;
}

static int64_t tiles_for(int64_t m, int64_t p, int tm, int tn) {
    return ((m + tm - 1) / tm) * ((p + tn - 1) / tn);
}

// Split-k chosen by the planner (MOA_FLAG_SPLIT_K absent): a product whose
// 128 x 128 blocks leave most of the 256 CUs idle (at most 64 blocks) and
// whose k walk is long (n >= 4096) gets about 512 workgroups, each summing
// at least 512 k (measured on 256 x 65536 x 256, 512 x 32768 x 512 and
// 1024 x 16384 x 1024: 3 to 12 times faster than one workgroup per block).
static int auto_split_k(int64_t m, int64_t n, int64_t p) {
    const int64_t tiles = tiles_for(m, p, 128, 128);
    if (tiles > 64 || n < 4096) return 1;
    int64_t c = (512 + tiles - 1) / tiles;
    c = std::min<int64_t>(std::min<int64_t>(c, n / 512), 255);
    return c >= 2 ? (int)c : 1;
}

static int split_k_of(const moa_gemm_desc &d, int64_t slabs) {
    const int req = split_k_requested(d);
    return split_k_chunks(req == 0 ? auto_split_k(d.m, d.n, d.p) : req, slabs);
}

moa_status make_plan(const moa_gemm_desc &d_in, Plan *out) {
    const moa_gemm_desc d = row_major_result(d_in);   // a column-major C is planned as C^T
    Plan pl;
    pl.path = resolve_path(d);
    const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
    pl.static_components = static_block_components(kL1Bytes, es, 3);
    const int forced = (int)((d.flags >> 8) & 0xFF) - 1;   // MOA_FLAG_VARIANT
    switch (pl.path) {
    case MOA_PATH_ONF: {
        pl.kernel = d.dtype == MOA_F64 ? K_ONF_F64 : K_ONF_F32;
        const int nv = onf_variant_count((moa_dtype)d.dtype);
        // the ring kernels read row-major operands with 32-bit offsets
        const int ring = onf_ring_variant((moa_dtype)d.dtype);
        const bool ring_ok = !has_col_operand(d) && onf_ring_fits((moa_dtype)d.dtype, d.n, d.p);
        int v = 0;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (ONF has %d)", forced, nv);
            if (forced == ring && !ring_ok)
                return fail(MOA_ERR_UNSUPPORTED, "the ONF ring variant takes row-major operands whose rows fit "
                            "32-bit offsets");
            v = forced;
        } else if ((v = tuned_variant(d, pl.path)) >= 0 && (v != ring || ring_ok)) {
            pl.tuned = true;
        } else if (ring_ok && [&] {
                       Plan r;
                       onf_variant_shape((moa_dtype)d.dtype, ring, &r);
                       return tiles_for(d.m, d.p, r.tile_m, r.tile_n) >= kNumCUs;
                   }()) {
            v = ring;
        } else {
            v = 0;
            // register-staged blocks: the largest that still gives every CU a
            // block; FP64 stops at 64 x 128 (its 128 x 128 block needs more
            // registers than two waves per SIMD allow and measured slower)
            const int top = d.dtype == MOA_F64 ? 2 : ring - 1;
            for (int c = top; c >= 0; --c) {
                Plan t;
                onf_variant_shape((moa_dtype)d.dtype, c, &t);
                if (tiles_for(d.m, d.p, t.tile_m, t.tile_n) >= kNumCUs) { v = c; break; }
            }
        }
        onf_variant_shape((moa_dtype)d.dtype, v, &pl);
        if ((d.m + pl.tile_m - 1) / pl.tile_m > 65535)
            return fail(MOA_ERR_SHAPE, "m = %lld exceeds the ONF grid limit", (long long)d.m);
        break;
    }
    case MOA_PATH_MFMA_F32: {
        pl.kernel = K_MFMA_F32;
        const int nv = mfma_f32_variant_count();
        int v;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (MFMA_F32 has %d)", forced, nv);
            v = forced;
        } else if ((v = tuned_variant(d, pl.path)) >= 0 && !(has_col_operand(d) && v == mfma_f32_staged_variant())) {
            pl.tuned = true;
        } else {
            v = mfma_f32_default_variant(d.m, d.p);
        }
        // the register-staged kernel reads row-major operands only; the ring
        // variants condition a column-major operand with the other packer
        if (v == mfma_f32_staged_variant() && has_col_operand(d))
            return fail(MOA_ERR_UNSUPPORTED, "the register-staged FP32 variant takes row-major operands only");
        mfma_f32_shape(v, &pl);
        pl.workspace_bytes = mfma_f32_workspace_bytes(d.m, d.n, d.p, v);
        // the record ring's 32-bit offsets inside a row tile, as on split-BF16
        if (pl.workspace_bytes > 0 && (d.n + 15) / 16 > 131071)
            return fail(MOA_ERR_SHAPE, "n = %lld exceeds the FP32 record offset range", (long long)d.n);
        break;
    }
    case MOA_PATH_SPLIT_BF16: {
        pl.kernel = K_SPLIT_BF16;
        const int nv = split_bf16_variant_count();
        int v = 0;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (SPLIT_BF16 has %d)", forced, nv);
            v = forced;
        } else if ((v = tuned_variant(d, pl.path)) >= 0) {
            pl.tuned = true;
        } else {
            v = split_bf16_default_variant(d.m, d.p);
        }
        split_bf16_shape(v, &pl);
        pl.workspace_bytes = split_bf16_workspace_bytes(d.m, d.n, d.p);
        pl.split_k = split_k_of(d, (d.n + 15) / 16);
        if (pl.split_k > 1) split_bf16_shape(0, &pl);   // split-k runs the first block variant
        // 256 record rows of (n/16) 64-byte records must stay below 2^31 bytes
        // (32-bit buffer offsets of one tile).
        if ((d.n + 15) / 16 > 131071)
            return fail(MOA_ERR_SHAPE, "n = %lld exceeds the split-BF16 offset range", (long long)d.n);
        break;
    }
    case MOA_PATH_FP8_SCALED: {
        const bool two = fp8_two_term(d);
        pl.kernel = two ? K_FP8_2TERM : K_FP8;
        const int nv = fp8_variant_count(two);
        int v = 0;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (FP8 has %d)", forced, nv);
            v = forced;
        } else if ((v = tuned_variant(d, pl.path)) >= 0) {
            pl.tuned = true;
        } else {
            v = 0;
            for (int c = nv - 1; c >= 0; --c) {
                Plan t;
                fp8_shape(two, c, &t);
                if (tiles_for(d.m, d.p, t.tile_m, t.tile_n) >= kNumCUs) { v = c; break; }
            }
            if (!two) {
                // one term: when the 256 x 256 blocks fill more than one round of
                // the CUs but leave the last round less than 40% full, the
                // 128 x 128 blocks (three per CU) finish sooner (measured N = 6144:
                // 0.24 vs 0.27 ms, 7168: 0.40 vs 0.42 ms)
                Plan t;
                fp8_shape(two, v, &t);
                const int64_t big = tiles_for(d.m, d.p, t.tile_m, t.tile_n), tail = big % kNumCUs;
                if (t.tile_m == 256 && big > kNumCUs && tail != 0 && 10 * tail < 4 * kNumCUs) v = 0;
            }
        }
        fp8_shape(two, v, &pl);
        pl.workspace_bytes = fp8_workspace_bytes(d.m, d.n, d.p, two);
        pl.split_k = split_k_of(d, (d.n + 63) / 64);
        if (pl.split_k > 1) fp8_shape(two, 0, &pl);     // split-k runs the first block variant
        // 256 record rows of (n/64) 64-byte records must stay below 2^31 bytes
        // (32-bit buffer offsets of one tile).
        if ((d.n + 63) / 64 > 131071)
            return fail(MOA_ERR_SHAPE, "n = %lld exceeds the FP8 offset range", (long long)d.n);
        break;
    }
    default:
        return fail(MOA_ERR_INVALID, "unknown path %d", d.path);
    }
    pl.workgroups = tiles_for(d.m, d.p, pl.tile_m, pl.tile_n);
    if (pl.split_k > 1) {
        // the partials follow the path's own workspace, 256-byte aligned
        pl.partial_offset = (pl.workspace_bytes + 255) / 256 * 256;
        int64_t mp = 0;
        if (__builtin_mul_overflow(d.m, d.p, &mp) || mp > (INT64_MAX / 4) / pl.split_k)
            return fail(MOA_ERR_SHAPE, "split-k partials overflow");
        pl.workspace_bytes = pl.partial_offset + (int64_t)pl.split_k * mp * 4;
        pl.workgroups *= pl.split_k;
    }
    if (pl.workgroups > INT32_MAX) return fail(MOA_ERR_SHAPE, "too many tiles");
    *out = pl;
    return MOA_OK;
}

}  // namespace moa
