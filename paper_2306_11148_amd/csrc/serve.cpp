// Serving loop (placeholder until the scheduler lands).
#include "moa_internal.h"

using namespace moa;

struct moa_server {};

extern "C" {
moa_status moa_serve_create(const moa_serve_cfg *, moa_server **out) {
    if (out) *out = nullptr;
    return fail(MOA_ERR_UNSUPPORTED, "serving not built yet");
}
moa_status moa_serve_submit(moa_server *, const moa_gemm_desc *, uint64_t *) {
    return fail(MOA_ERR_UNSUPPORTED, "serving not built yet");
}
moa_status moa_serve_poll(moa_server *, uint64_t, moa_req_info *) {
    return fail(MOA_ERR_UNSUPPORTED, "serving not built yet");
}
moa_status moa_serve_drain(moa_server *) { return fail(MOA_ERR_UNSUPPORTED, "serving not built yet"); }
moa_status moa_serve_destroy(moa_server *) { return MOA_OK; }
}
