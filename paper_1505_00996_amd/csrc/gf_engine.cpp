// Batched launch and request interface (gf_fast_batched, gf_submit, gf_poll).
#include <hip/hip_runtime_api.h>

#include "gf_api_internal.h"

namespace gf {

gf_status engine_start(gf_ctx *, size_t, int) { return fail(GF_ENOTSUP, "request interface not built"); }
void engine_stop(gf_ctx *) {}

}  // namespace gf

using namespace gf;

extern "C" {

size_t gf_batched_workspace_bytes(int32_t, const gf_image *, const gf_image *, const gf_params *) { return 0; }

gf_status gf_fast_batched(gf_ctx *, int32_t, const gf_image *, const gf_image *, gf_image *,
                          const gf_params *, void *, size_t, void *) {
    return fail(GF_ENOTSUP, "batched launch not built");
}

gf_status gf_submit(gf_ctx *ctx, const gf_image *, const gf_image *, gf_image *, const gf_params *,
                    uint64_t *) {
    if (!ctx) return fail(GF_EINVAL, "gf_submit needs a context");
    return fail(GF_ENOTSUP, "request interface not built");
}

gf_status gf_poll(gf_ctx *ctx, uint64_t, int32_t, gf_req_stats *) {
    if (!ctx) return fail(GF_EINVAL, "gf_poll needs a context");
    return fail(GF_ENOTSUP, "request interface not built");
}

}  // extern "C"
