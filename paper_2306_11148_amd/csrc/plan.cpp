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
#include <cstdlib>

#include "moa_internal.h"

namespace moa {

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

moa_status make_plan(const moa_gemm_desc &d, Plan *out) {
    Plan pl;
    pl.path = resolve_path(d);
    const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
    pl.static_components = static_block_components(kL1Bytes, es, 3);
    const int forced = (int)((d.flags >> 8) & 0xFF) - 1;   // MOA_FLAG_VARIANT
    switch (pl.path) {
    case MOA_PATH_ONF: {
        pl.kernel = d.dtype == MOA_F64 ? K_ONF_F64 : K_ONF_F32;
        const int nv = onf_variant_count((moa_dtype)d.dtype);
        int v = 0;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (ONF has %d)", forced, nv);
            v = forced;
        } else {
            for (int c = nv - 1; c >= 0; --c) {
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
    case MOA_PATH_MFMA_F32:
        pl.kernel = K_MFMA_F32;
        if (forced > 0) return fail(MOA_ERR_INVALID, "variant %d out of range (MFMA_F32 has 1)", forced);
        mfma_f32_shape(&pl);
        break;
    case MOA_PATH_SPLIT_BF16: {
        pl.kernel = K_SPLIT_BF16;
        const int nv = split_bf16_variant_count();
        int v = 0;
        if (forced >= 0) {
            if (forced >= nv) return fail(MOA_ERR_INVALID, "variant %d out of range (SPLIT_BF16 has %d)", forced, nv);
            v = forced;
        } else {
            for (int c = nv - 1; c >= 0; --c) {
                Plan t;
                split_bf16_shape(c, &t);
                if (tiles_for(d.m, d.p, t.tile_m, t.tile_n) >= kNumCUs) { v = c; break; }
            }
        }
        split_bf16_shape(v, &pl);
        pl.workspace_bytes = split_bf16_workspace_bytes(d.m, d.n, d.p);
        // 256 record rows of (n/16) 64-byte records must stay below 2^31 bytes
        // (32-bit buffer offsets of one tile).
        if ((d.n + 15) / 16 > 131071)
            return fail(MOA_ERR_SHAPE, "n = %lld exceeds the split-BF16 offset range", (long long)d.n);
        break;
    }
    case MOA_PATH_FP8_SCALED: {
        const bool two = (d.flags & MOA_FLAG_FP8_TWO_TERM) != 0;
        pl.kernel = two ? K_FP8_2TERM : K_FP8;
        if (forced > 0) return fail(MOA_ERR_INVALID, "variant %d out of range (FP8 has 1)", forced);
        fp8_shape(two, &pl);
        pl.workspace_bytes = fp8_workspace_bytes(d.m, d.n, d.p, two);
        break;
    }
    default:
        return fail(MOA_ERR_INVALID, "unknown path %d", d.path);
    }
    pl.workgroups = tiles_for(d.m, d.p, pl.tile_m, pl.tile_n);
    if (pl.workgroups > INT32_MAX) return fail(MOA_ERR_SHAPE, "too many tiles");
    *out = pl;
    return MOA_OK;
}

}  // namespace moa
