// Context lifetime, device selection and per-context tile choices.
#include <hip/hip_runtime_api.h>

#include <new>

#include "gf_api_internal.h"

namespace gf {

gf_status ctx_use_device(gf_ctx *ctx) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return fail(GF_EDEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
    }
    return GF_OK;
}

// Problem class of a tuned choice: dtype, channels, s, low-res radius and
// the size class floor(log2(Hl * Wl)).
uint64_t tile_key(gf_dtype dt, int h, int w, int C, int r, int s) {
    const int R = lowres_radius(r, s);
    const uint64_t n = (uint64_t)((h + s - 1) / s) * (uint64_t)((w + s - 1) / s);
    int lg = 0;
    while ((n >> (lg + 1)) != 0) ++lg;
    return ((uint64_t)(dt & 0xf) << 60) | ((uint64_t)(C & 0xfff) << 48) |
           ((uint64_t)(s & 0xffff) << 32) | ((uint64_t)(R & 0xffffff) << 8) | (uint64_t)(lg & 0xff);
}

bool ctx_tiles(gf_ctx *ctx, const gf_image *I, const gf_image *p, const gf_params *pr, TileCfg *out) {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    auto it = ctx->tuned.find(tile_key(I->dtype, I->h, I->w, p->c, pr->r, pr->s));
    if (it == ctx->tuned.end()) return false;
    *out = it->second;
    return true;
}

static hipEvent_t take_event(gf_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(gf_ctx *c, int k, hipStream_t s, bool in_disp)
    : ctx(c), kernel(k), st(s), in_dispatch(in_disp) {
    if (!ctx || !ctx->profiling) return;
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    start = take_event(ctx);
    if (!start) return;
    if (in_dispatch) {
        end = take_event(ctx);
        if (!end) {
            ctx->event_pool.push_back(start);
            start = nullptr;
        }
    } else if (hipEventRecord(start, st) != hipSuccess) {
        ctx->event_pool.push_back(start);
        start = nullptr;
    }
}

ProfScope::~ProfScope() {
    if (!start) return;
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    if (in_dispatch) {
        if (committed) {
            ctx->marks.push_back({kernel, start, end});
        } else {
            ctx->event_pool.push_back(start);
            ctx->event_pool.push_back(end);
        }
        return;
    }
    end = take_event(ctx);
    if (end && hipEventRecord(end, st) == hipSuccess) {
        ctx->marks.push_back({kernel, start, end});
    } else {
        ctx->event_pool.push_back(start);
        if (end) ctx->event_pool.push_back(end);
    }
}

}  // namespace gf

using namespace gf;

extern "C" {

gf_status gf_ctx_create(gf_ctx **out, int device, size_t arena_bytes, int max_inflight) {
    if (!out) return fail(GF_EINVAL, "out is NULL");
    *out = nullptr;
    if (device < 0) return fail(GF_EINVAL, "device %d < 0", device);
    if (max_inflight < 0) return fail(GF_EINVAL, "max_inflight %d < 0", max_inflight);
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(GF_EDEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (device >= n) return fail(GF_EINVAL, "device %d of %d", device, n);
    gf_ctx *ctx = new (std::nothrow) gf_ctx;
    if (!ctx) return fail(GF_ENOMEM, "out of host memory");
    ctx->device = device;
    gf_status st = ctx_use_device(ctx);
    if (st == GF_OK) st = noalloc_prepare();
    if (st == GF_OK && arena_bytes > 0) st = engine_start(ctx, arena_bytes, max_inflight ? max_inflight : 64);
    if (st != GF_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return GF_OK;
}

gf_status gf_ctx_set_fusion(gf_ctx *ctx, gf_fusion mode) {
    if (!ctx) return fail(GF_EINVAL, "gf_ctx_set_fusion needs a context");
    if (mode != GF_FUSE_OFF && mode != GF_FUSE_AUTO && mode != GF_FUSE_ON)
        return fail(GF_EINVAL, "unknown fusion mode %d", (int)mode);
    ctx->fuse.store((int)mode);
    return GF_OK;
}

gf_status gf_ctx_profile(gf_ctx *ctx, int enable) {
    if (!ctx) return fail(GF_EINVAL, "gf_ctx_profile needs a context");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->profiling = enable != 0;
    return GF_OK;
}

gf_status gf_ctx_profile_read(gf_ctx *ctx, gf_kernel_time *out) {
    if (!ctx || !out) return fail(GF_EINVAL, "gf_ctx_profile_read: null argument");
    std::vector<gf_ctx::Mark> marks;
    {
        std::lock_guard<std::mutex> lk(ctx->prof_mu);
        marks.swap(ctx->marks);
    }
    for (int k = 0; k < GF_NKERNELS; ++k) out[k] = gf_kernel_time{0.0, 0};
    gf_status st = GF_OK;
    for (auto &m : marks) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(m.end);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.start, m.end);
        if (e != hipSuccess) {
            st = fail(GF_EDEVICE, "event timing: %s", hipGetErrorString(e));
        } else {
            out[m.kernel].total_ms += ms;
            out[m.kernel].launches += 1;
        }
    }
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &m : marks) {
        ctx->event_pool.push_back(m.start);
        ctx->event_pool.push_back(m.end);
    }
    return st;
}

void gf_ctx_destroy(gf_ctx *ctx) {
    if (!ctx) return;
    (void)ctx_use_device(ctx);
    engine_stop(ctx);
    {
        std::lock_guard<std::mutex> lk(ctx->prof_mu);
        for (auto &m : ctx->marks) {
            (void)hipEventSynchronize(m.end);
            ctx->event_pool.push_back(m.start);
            ctx->event_pool.push_back(m.end);
        }
        ctx->marks.clear();
        for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
        ctx->event_pool.clear();
    }
    if (ctx->ws || ctx->pin) (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    if (ctx->pin_ev) (void)hipEventDestroy(ctx->pin_ev);
    delete ctx;
}

}  // extern "C"
