// sk_scale without device allocation: the same scaling path as sk_scale, with
// its working memory carved from a file-scope device array (`scratch`) that
// the library holds on every GPU it runs on, instead of the caller's arena.
//
// The array's name is a host-side stand-in in host code; the device address
// of each GPU's copy is resolved once per device by static_scratch_init
// (called by sk_create with that device current) and only that address is
// passed on (Bump base -> kernel arguments, copies).
#include <mutex>

#include "sk_runtime.h"

namespace sk {

static __device__ __align__(256) char scratch[SK_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

}  // namespace sk

using namespace sk;

sk_status sk_scale_static(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                          void *potentials, sk_report *report) {
    if (!ctx) return SK_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!params) return fail(ctx, SK_EINVAL, "params is NULL");
    if (const sk_status st = check_size(ctx, n, params); st != SK_OK) return st;
    const size_t need = sk_arena_bytes(n, params->storage);
    if (need > (size_t)SK_STATIC_SCRATCH_BYTES)
        return fail(ctx, SK_ENOMEM,
                    "n = %d with storage %d needs %zu bytes of working memory; the static "
                    "scratch holds %zu (use sk_scale with an arena)",
                    n, params->storage, need, (size_t)SK_STATIC_SCRATCH_BYTES);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> gs(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) ptr = g_scratch_ptr[ctx->device];
    }
    if (!ptr) return fail(ctx, SK_EDEVICE, "static scratch not resolved on device %d", ctx->device);
    const int16_t *Ws[1] = {W};
    void *pots[1] = {potentials};
    return scale_impl(ctx, 1, Ws, &n, params, pots, report, (char *)ptr,
                      (size_t)SK_STATIC_SCRATCH_BYTES);
}
