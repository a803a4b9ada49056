// Served path (continuous batching): placeholder until the scheduler lands.
#include "sk_runtime.h"

namespace sk {
void serve_stop(sk_ctx *) {}
}  // namespace sk

extern "C" sk_status sk_submit(sk_ctx *ctx, const int16_t *, int32_t, const sk_params *, uint64_t *) {
    if (!ctx) return SK_EINVAL;
    return sk::fail(ctx, SK_EINVAL, "serving is not available in this build");
}
extern "C" sk_status sk_poll(sk_ctx *ctx, uint64_t, int32_t *, int64_t *, sk_report *) {
    if (!ctx) return SK_EINVAL;
    return sk::fail(ctx, SK_EINVAL, "serving is not available in this build");
}
