// Grouped products (placeholder: members run one after another on the
// stream; replaced by the persistent grouped kernel).
#include "moa_internal.h"

using namespace moa;

extern "C" moa_status moa_gemm_grouped(const moa_gemm_desc *descs, int64_t count, void *stream) {
    if (count < 0) return fail(MOA_ERR_INVALID, "negative count");
    if (count > 0 && !descs) return fail(MOA_ERR_INVALID, "null descriptor array");
    for (int64_t g = 0; g < count; ++g) {
        moa_status s = validate(descs[g], true);
        if (s != MOA_OK) return s;
    }
    for (int64_t g = 0; g < count; ++g) {
        moa_status s = run_gemm(descs[g], static_cast<hipStream_t>(stream));
        if (s != MOA_OK) return s;
    }
    return MOA_OK;
}
