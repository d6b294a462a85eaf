// gf_fast_noalloc: the Fast Guided Filter (Algorithm 2) for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// that forbid allocation).  It runs the kernels of gf_fast with the
// low-resolution maps (a, b, their box means and, with area subsampling, the
// subsampled I' and p') in `scratch`, a fixed array in device memory that
// lives as long as the process, instead of a workspace.
//
// In host code the name `scratch` stands for a host-side shadow, not for a
// device address: it must never be handed to a kernel or a copy.  The device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (at gf_ctx_create for the context's device, else on the
// first call made with that device current) and only that address is used.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "gf_api_internal.h"

namespace {

constexpr size_t kScratchBytes = GF_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lookup_mu;                       // serialises the first lookup per device
std::atomic<void *> g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's `scratch`, looked up on first use.
gf_status scratch_on_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gf::fail(GF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return gf::fail(GF_ENOTSUP, "gf_fast_noalloc: device %d above the %d devices it serves", dev, kMaxDevices);
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lk(g_lookup_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return gf::fail(GF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                hipGetErrorString(e));
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return GF_OK;
}

}  // namespace

namespace gf {

// Called by gf_ctx_create with the context's device current.
gf_status noalloc_prepare() {
    void *p = nullptr;
    return scratch_on_current_device(&p);
}

}  // namespace gf

extern "C" gf_status gf_fast_noalloc(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                                     const gf_params *pr, void *stream) {
    using namespace gf;
    gf_status st = validate(I, p, q, pr);
    if (st != GF_OK) return st;
    const Geo g = make_geo(I->h, I->w, p->c, *pr, I->c);
    const size_t need = workspace_bytes(g);
    if (need > kScratchBytes)
        return fail(GF_ENOMEM, "gf_fast_noalloc: the low-res maps of this call need %zu bytes, above the %zu-byte "
                    "fixed scratch array (use gf_fast with a workspace)", need, kScratchBytes);
    if (ctx && (st = ctx_use_device(ctx)) != GF_OK) return st;
    void *ws = nullptr;
    if ((st = scratch_on_current_device(&ws)) != GF_OK) return st;
    TileCfg tuned;
    const bool have = ctx && ctx_tiles(ctx, I, p, pr, &tuned);
    // no context into run_fast: its profiling events are not taken here
    return run_fast(nullptr, I, p, q, pr, ws, kScratchBytes, (hipStream_t)stream, have ? &tuned : nullptr);
}
