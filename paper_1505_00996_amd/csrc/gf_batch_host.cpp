// Host side of the persistent batched launch: planning (task queue layout,
// workspace layout, tile height) and gf_fast_batched / gf_batched_workspace_bytes.
#include <hip/hip_runtime_api.h>

#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "gf_api_internal.h"
#include "gf_batch_host.h"

namespace gf {

static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Tile height shared by every image of the launch: the requested one, else
// 24, falling back to smaller heights until the staged tiles of the batch's
// largest r' fit in LDS (the queue kernel also holds the output patch and a
// few static words); 0 when none fits (the batch then runs as per-image
// launches).  The choice depends only on the configuration and the largest
// radius, so an image gives the same bits alone and in any batch, and the
// same bits as gf_fast with tiles {th, thb}.  Box-mean tiles (thb) are 48
// rows under the phase schedule wherever they fit in LDS (on the 256-image
// mix the box phase took 446 us at 48 rows against 561 us at 24, while the
// coefficient phase is fastest at 24), else th.
static int batch_thb(int sched, int th, int maxR) {
    if (sched == GF_BATCH_PHASES && box_lds_bytes(TileCfg{th, 48}, maxR) <= kLdsLimit) return 48;
    return th;
}

static int batch_th(int sched, int want, int maxR, BatchPlan *plan) {
    // 32 and 48 rows only when asked for, and for the phase schedule only
    // (the queue kernel carries every phase's LDS and registers at once)
    const int cap = std::min(want ? want : 24, sched == GF_BATCH_QUEUE ? 24 : 48);
    for (int th : {48, 32, 24, 16, 8}) {
        if (th > cap) continue;
        const TileCfg t{th, batch_thb(sched, th, maxR)};
        if (!coeff_staged(t, maxR)) continue;
        const size_t c = coeff_lds_bytes(t, maxR), b = box_lds_bytes(t, maxR);
        if (sched == GF_BATCH_QUEUE) {
            const size_t all = std::max({c, b, kOutPatchLds});
            if (all + 256 > kLdsLimit) continue;
            plan->lds = all;
        } else if (c > kLdsLimit || b > kLdsLimit) {
            continue;
        }
        plan->lds_coeff = c;
        plan->lds_box = b;
        plan->thb = t.box_th;
        return th;
    }
    return 0;
}

TileCfg batch_tiles(const gf_batch_cfg &cfg, int maxR) {
    BatchPlan scratch;
    const int th = batch_th(cfg.schedule, cfg.tile_h, maxR, &scratch);
    return TileCfg{th, th ? scratch.thb : 0};
}

static bool cfg_ok(const gf_batch_cfg &c) {
    return (c.schedule == GF_BATCH_PHASES || c.schedule == GF_BATCH_QUEUE) &&
           (c.tile_h == 0 || c.tile_h == 8 || c.tile_h == 16 || c.tile_h == 24 || c.tile_h == 32 ||
            c.tile_h == 48);
}

gf_batch_cfg ctx_batch_cfg(gf_ctx *ctx) {
    if (!ctx) return gf_batch_cfg{GF_BATCH_PHASES, 0};
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    return ctx->batch_cfg;
}

bool batch_cfg_ok(const gf_batch_cfg &c) { return cfg_ok(c); }

gf_status plan_batch(int n, const gf_image *I, const gf_image *p, const gf_image *q,
                     const gf_params *pr, char *ws_base, const gf_batch_cfg &cfg, BatchPlan *plan) {
    if (n < 1) return fail(GF_EINVAL, "batch of %d images", n);
    if (!cfg_ok(cfg)) return fail(GF_EINVAL, "batch configuration {%d, %d}", cfg.schedule, cfg.tile_h);
    if (!I || !p || !q || !pr) return fail(GF_EINVAL, "batch: null array");
    gf_status st;
    int maxR = 0;
    bool per_image = false;
    for (int i = 0; i < n; ++i) {
        if ((st = validate(&I[i], &p[i], &q[i], &pr[i])) != GF_OK)
            return fail(st, "image %d: %s", i, last_error());
        if (I[i].dtype != I[0].dtype) return fail(GF_EINVAL, "image %d: dtype differs from image 0", i);
        maxR = std::max(maxR, lowres_radius(pr[i].r, pr[i].s));
        per_image = per_image || (pr[i].sub == GF_SUB_AREA && pr[i].s > 1) || I[i].c == 3;
    }
    plan->n = n;
    plan->dtype = I[0].dtype;
    plan->sched = cfg.schedule;
    // area subsampling has a pass of its own and a colour guide kernels of
    // its own that the batched kernels do not run: such a batch goes image
    // by image
    plan->th = per_image ? 0 : batch_th(cfg.schedule, cfg.tile_h, maxR, plan);
    plan->desc.assign(n, BDesc{});
    // plan order: by ratio class (stable), so each class's output blocks are contiguous
    plan->order.resize(n);
    for (int k = 0; k < n; ++k) plan->order[k] = k;
    std::stable_sort(plan->order.begin(), plan->order.end(),
                     [&](int a, int b) { return ratio_class(pr[a].s) < ratio_class(pr[b].s); });
    // workspace: control words, descriptor table, then each image's 4C planes
    // (and its 1 + C area-subsampled planes)
    size_t off = round256(sizeof(unsigned) * batch_ctl_words(n));
    plan->desc_off = off;
    off += round256(sizeof(BDesc) * n);
    unsigned base[3] = {0, 0, 0};
    for (int k = 0; k < n; ++k) {
        const int i = plan->order[k];
        BDesc &d = plan->desc[k];
        const Geo g = make_geo(I[i].h, I[i].w, p[i].c, pr[i], I[i].c);
        d.I = I[i].data;
        d.P = p[i].data;
        d.Q = q[i].data;
        d.Irs = I[i].row_stride;
        d.Prs = p[i].row_stride;
        d.Pps = p[i].plane_stride;
        d.Qrs = q[i].row_stride;
        d.Qps = q[i].plane_stride;
        d.g = g;
        d.kind = (g.s == 1 || area_pass(g)) ? 0 : ((g.sub == GF_SUB_NEAREST || (g.s & 1)) ? 1 : 2);
        const int th = plan->th ? plan->th : 8, thb = plan->th ? plan->thb : 8;
        d.ntx_l = (g.Wl + kTileW - 1) / kTileW;
        d.nty_l = (g.Hl + th - 1) / th;
        d.nty_b = (g.Hl + thb - 1) / thb;
        const int ow = 64 * out_px(cfg.schedule, I[0].dtype);
        d.ntx_o = (g.W + ow - 1) / ow;
        d.nty_o = (g.H + 4 * 8 - 1) / (4 * 8);
        d.ntiles[0] = (unsigned)(d.ntx_l * d.nty_l);  // a coefficient task covers every channel
        d.ntiles[1] = (unsigned)(d.ntx_l * d.nty_b * 2 * g.C);
        d.ntiles[2] = (unsigned)(d.ntx_o * d.nty_o * ((g.C + 2) / 3));
        // the image's workspace as gf_fast lays it out: a, b planes, their box
        // means right after them (the batched kernels' layout), then any
        // area-subsampled planes
        // (no addresses when only sizes are asked for: ws_base null)
        d.coef = ws_base ? (float *)(ws_base + off) : nullptr;
        d.mean = ws_base ? d.coef + (size_t)g.lps * 2 * g.C : nullptr;
        off += round256(workspace_bytes(g));
        for (int ph = 0; ph < 3; ++ph) {
            d.base[ph] = base[ph];
            base[ph] += d.ntiles[ph];
        }
    }
    // phases follow each other in the queue
    for (int k = 0; k < n; ++k) {
        plan->desc[k].base[1] += base[0];
        plan->desc[k].base[2] += base[0] + base[1];
    }
    for (int c = 0; c < kRatioClasses; ++c) plan->out.lo[c] = plan->out.hi[c] = 0;
    for (int k = n - 1; k >= 0; --k) {  // each class's first image sets lo, its last sets hi
        const BDesc &d = plan->desc[k];
        const int c = ratio_class(d.g.s);
        plan->out.lo[c] = d.base[2];
        if (plan->out.hi[c] == 0) plan->out.hi[c] = d.base[2] + d.ntiles[2];
    }
    plan->p1 = base[0];
    plan->p2 = base[0] + base[1];
    plan->total = base[0] + base[1] + base[2];
    plan->ws_bytes = off;
    return GF_OK;
}

// Workgroups of the persistent launch: as many as can be resident at once,
// never more than there are tasks.
static int plan_grid(const BatchPlan &plan) {
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    const int occ = batched_occupancy(plan.dtype, plan.th, plan.lds);
    return (int)std::min<unsigned>(plan.total, (unsigned)(occ * ncu));
}

static gf_status enqueue_plan(gf_ctx *ctx, const BatchPlan &plan, void *ws, int grid, bool set_lds,
                              unsigned spin_limit, hipStream_t st) {
    char *base = (char *)ws;
    const BDesc *D = (const BDesc *)(base + plan.desc_off);
    ProfScope ps(ctx, GF_K_BATCHED, st);
    const hipError_t e =
        plan.sched == GF_BATCH_QUEUE
            ? launch_batched(plan.dtype, plan.th, D, plan.n, (unsigned *)base, plan.total, plan.p1, plan.p2,
                             plan.lds, grid, set_lds, spin_limit, st)
            : launch_phases(plan.dtype, plan.th, plan.thb, D, plan.n, (unsigned *)base, plan.p1, plan.p2, plan.out,
                            plan.lds_coeff, plan.lds_box, set_lds, st);
    if (e != hipSuccess) return fail(GF_EDEVICE, "batched launch: %s", hipGetErrorString(e));
    return GF_OK;
}

gf_status launch_plan(gf_ctx *ctx, BatchPlan &plan, void *ws, hipStream_t st) {
    char *base = (char *)ws;
    const size_t dbytes = sizeof(BDesc) * plan.n;
    // The descriptor table goes through pinned host memory owned by the
    // context (reused once the previous upload from it has completed), or,
    // without a context, through a temporary buffer and a stream sync.
    hipError_t e;
    if (ctx) {
        std::lock_guard<std::mutex> lk(ctx->pin_mu);
        if (ctx->pin_ev) (void)hipEventSynchronize(ctx->pin_ev);
        if (ctx->pin_bytes < dbytes) {
            if (ctx->pin) (void)hipHostFree(ctx->pin);
            ctx->pin = nullptr;
            ctx->pin_bytes = 0;
            if ((e = hipHostMalloc(&ctx->pin, dbytes, hipHostMallocDefault)) != hipSuccess)
                return fail(GF_ENOMEM, "hipHostMalloc(%zu): %s", dbytes, hipGetErrorString(e));
            ctx->pin_bytes = dbytes;
        }
        if (!ctx->pin_ev && (e = hipEventCreateWithFlags(&ctx->pin_ev, hipEventDisableTiming)) != hipSuccess)
            return fail(GF_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        memcpy(ctx->pin, plan.desc.data(), dbytes);
        e = hipMemcpyAsync(base + plan.desc_off, ctx->pin, dbytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(ctx->pin_ev, st);
    } else {
        e = hipMemcpyAsync(base + plan.desc_off, plan.desc.data(), dbytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) return fail(GF_EDEVICE, "descriptor upload: %s", hipGetErrorString(e));
    return enqueue_plan(ctx, plan, ws, plan_grid(plan), true, ctx ? ctx->spin_limit.load() : kBatchSpinLimit, st);
}

}  // namespace gf

using namespace gf;

// A planned batch whose launch needs no host work beyond kernel enqueues.
struct gf_batch {
    int device = 0;
    BatchPlan plan;
    void *ws = nullptr;
    int grid = 0;
    unsigned spin_limit = kBatchSpinLimit;  // the context's at creation
    // per-image launches (plan.th == 0): the problems as given
    std::vector<gf_image> I, p, q;
    std::vector<gf_params> pr;
};

extern "C" {

size_t gf_batched_workspace_bytes(int32_t n, const gf_image *I, const gf_image *p,
                                  const gf_params *pr) {
    if (n < 1 || !I || !p || !pr) return 0;
    size_t planes = 0;
    for (int i = 0; i < n; ++i) {
        if (I[i].h < 1 || I[i].w < 1 || p[i].c < 1 || pr[i].s < 1 || pr[i].r < 0) return 0;
        if (I[i].c != 1 && I[i].c != 3) return 0;
        planes += round256(workspace_bytes(make_geo(I[i].h, I[i].w, p[i].c, pr[i], I[i].c)));
    }
    return round256(sizeof(unsigned) * batch_ctl_words(n)) + round256(sizeof(BDesc) * n) + planes;
}

size_t gf_footprint_bytes(int32_t h, int32_t w, int32_t c, gf_dtype dtype, const gf_params *pr) {
    if (!pr || (dtype != GF_F32 && dtype != GF_F16 && dtype != GF_BF16)) return 0;
    gf_image I{nullptr, dtype, 1, h, w, w, (int64_t)w * h};
    gf_image p{nullptr, dtype, c, h, w, w, (int64_t)w * h};
    return gf_batched_workspace_bytes(1, &I, &p, pr);
}

gf_status gf_fast_batched(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p, gf_image *q,
                          const gf_params *pr, void *ws, size_t ws_bytes, void *stream) {
    gf_status st;
    BatchPlan plan;
    const gf_batch_cfg cfg = ctx_batch_cfg(ctx);
    if ((st = plan_batch(n, I, p, q, pr, (char *)ws, cfg, &plan)) != GF_OK) return st;
    if (ctx && (st = ctx_use_device(ctx)) != GF_OK) return st;
    if (!ws) {
        if (!ctx) return fail(GF_EINVAL, "workspace is NULL and there is no context");
        if ((st = ctx_workspace(ctx, plan.ws_bytes, &ws)) != GF_OK) return st;
        if ((st = plan_batch(n, I, p, q, pr, (char *)ws, cfg, &plan)) != GF_OK) return st;
    } else if (ws_bytes < plan.ws_bytes) {
        return fail(GF_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, plan.ws_bytes);
    }
    if ((uintptr_t)ws % 256) return fail(GF_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (plan.th == 0) {
        // radius too large for the persistent kernel's staged tiles, area
        // subsampling or a colour guide: one gf_fast per image on the same
        // stream (same results)
        for (int k = 0; k < n; ++k) {
            const BDesc &d = plan.desc[k];
            const int i = plan.order[k];
            if ((st = run_fast(ctx, &I[i], &p[i], &q[i], &pr[i], d.coef, workspace_bytes(d.g), s, nullptr)) !=
                GF_OK)
                return st;
        }
        return GF_OK;
    }
    return launch_plan(ctx, plan, ws, s);
}

gf_status gf_batch_create(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p, gf_image *q,
                          const gf_params *pr, void *ws, size_t ws_bytes, void *stream, gf_batch **out) {
    if (!out) return fail(GF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ws) return fail(GF_EINVAL, "a prepared batch needs a caller-owned workspace");
    if ((uintptr_t)ws % 256) return fail(GF_EINVAL, "workspace not 256-byte aligned");
    gf_status st;
    if (ctx && (st = ctx_use_device(ctx)) != GF_OK) return st;
    gf_batch *b = new (std::nothrow) gf_batch;
    if (!b) return fail(GF_ENOMEM, "host allocation");
    if ((st = plan_batch(n, I, p, q, pr, (char *)ws, ctx_batch_cfg(ctx), &b->plan)) != GF_OK) {
        delete b;
        return st;
    }
    if (ws_bytes < b->plan.ws_bytes) {
        const size_t need = b->plan.ws_bytes;
        delete b;
        return fail(GF_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    }
    (void)hipGetDevice(&b->device);
    b->ws = ws;
    if (ctx) b->spin_limit = ctx->spin_limit.load();
    hipStream_t s = (hipStream_t)stream;
    if (b->plan.th == 0) {
        b->I.assign(I, I + n);
        b->p.assign(p, p + n);
        b->q.assign(q, q + n);
        b->pr.assign(pr, pr + n);
    } else {
        hipError_t e = hipMemcpyAsync((char *)ws + b->plan.desc_off, b->plan.desc.data(),
                                      sizeof(BDesc) * n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = b->plan.sched == GF_BATCH_QUEUE
                    ? batched_allow_lds(b->plan.dtype, b->plan.th, b->plan.lds)
                    : phases_allow_lds(b->plan.dtype, b->plan.th, b->plan.thb, b->plan.lds_coeff, b->plan.lds_box);
        if (e != hipSuccess) {
            delete b;
            return fail(GF_EDEVICE, "descriptor upload: %s", hipGetErrorString(e));
        }
        b->grid = plan_grid(b->plan);
    }
    *out = b;
    return GF_OK;
}

gf_status gf_batch_launch(const gf_batch *b, void *stream) {
    if (!b) return fail(GF_EINVAL, "batch is NULL");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != b->device) {
        const hipError_t e = hipSetDevice(b->device);
        if (e != hipSuccess) return fail(GF_EDEVICE, "hipSetDevice(%d): %s", b->device, hipGetErrorString(e));
    }
    hipStream_t s = (hipStream_t)stream;
    if (b->plan.th == 0) {
        gf_status st;
        for (int k = 0; k < b->plan.n; ++k) {
            const BDesc &d = b->plan.desc[k];
            const int i = b->plan.order[k];
            if ((st = run_fast(nullptr, &b->I[i], &b->p[i], const_cast<gf_image *>(&b->q[i]), &b->pr[i],
                               d.coef, workspace_bytes(d.g), s, nullptr)) != GF_OK)
                return st;
        }
        return GF_OK;
    }
    return enqueue_plan(nullptr, b->plan, b->ws, b->grid, false, b->spin_limit, s);
}

void gf_batch_destroy(gf_batch *b) { delete b; }

gf_status gf_ctx_set_wait_limit(gf_ctx *ctx, int64_t polls) {
    if (!ctx) return fail(GF_EINVAL, "ctx is NULL");
    if (polls > (int64_t)UINT32_MAX) return fail(GF_EINVAL, "wait limit %lld above 2^32 - 1", (long long)polls);
    ctx->spin_limit = polls < 0 ? kBatchSpinLimit : (uint32_t)polls;
    return GF_OK;
}

gf_status gf_ctx_set_batch_cfg(gf_ctx *ctx, const gf_batch_cfg *cfg) {
    if (!ctx) return fail(GF_EINVAL, "ctx is NULL");
    const gf_batch_cfg c = cfg ? *cfg : gf_batch_cfg{GF_BATCH_PHASES, 0};
    if (!cfg_ok(c)) return fail(GF_EINVAL, "batch configuration {%d, %d}", c.schedule, c.tile_h);
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->batch_cfg = c;
    return GF_OK;
}

}  // extern "C"
