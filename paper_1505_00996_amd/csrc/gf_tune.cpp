// Tile-shape autotuner for the window-sum kernels, pinned shapes, and their
// JSON cache (gf_ctx_set_tiles, gf_tune, gf_ctx_save_tuning,
// gf_ctx_load_tuning); the batch autotuner (gf_tune_batched).
#include <hip/hip_runtime_api.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gf_api_internal.h"
#include "gf_batch_host.h"

namespace gf {

static TileCfg from_abi(const gf_tiles &t) { return TileCfg{t.coeff_th, t.box_th}; }

static gf_tiles to_abi(const TileCfg &c) { return gf_tiles{c.coeff_th, c.box_th}; }

// Candidates of one kernel; the other kernel's field is taken from `base`.
static std::vector<TileCfg> candidates(const Geo &g, const TileCfg &base, int kernel) {
    std::vector<TileCfg> out;
    for (int th : {8, 16, 24, 32, 48, 64}) {
        TileCfg c = base;
        (kernel == GF_K_COEFF ? c.coeff_th : c.box_th) = th;
        if (tiles_fit(g, c)) out.push_back(c);
    }
    return out;
}

}  // namespace gf

using namespace gf;

extern "C" {

gf_status gf_ctx_set_tiles(gf_ctx *ctx, gf_dtype dtype, int32_t h, int32_t w, int32_t c,
                           const gf_params *pr, const gf_tiles *tiles) {
    if (!ctx || !pr) return fail(GF_EINVAL, "gf_ctx_set_tiles: null argument");
    if (h < 1 || w < 1 || c < 1 || pr->s < 1 || pr->r < 0)
        return fail(GF_EINVAL, "gf_ctx_set_tiles: bad problem size");
    const uint64_t key = tile_key(dtype, h, w, c, pr->r, pr->s);
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    if (!tiles) {
        ctx->tuned.erase(key);
        return GF_OK;
    }
    const Geo g = make_geo(h, w, c, *pr);
    const TileCfg t = from_abi(*tiles);
    if (!tiles_fit(g, t)) return fail(GF_ENOTSUP, "tile shapes do not fit r'=%d", g.R);
    ctx->tuned[key] = t;
    return GF_OK;
}

gf_status gf_tune(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                  const gf_params *pr, void *ws, size_t ws_bytes, void *stream, int32_t reps,
                  gf_tiles *best, gf_tune_result *results, int32_t max_results, int32_t *n_results) {
    if (!ctx) return fail(GF_EINVAL, "gf_tune needs a context");
    gf_status st = validate(I, p, q, pr);
    if (st != GF_OK) return st;
    if ((st = ctx_use_device(ctx)) != GF_OK) return st;
    if (reps < 1) reps = 1;
    if (I->c != 1) return fail(GF_ENOTSUP, "gf_tune covers the gray-guide kernels");
    const Geo g = make_geo(I->h, I->w, p->c, *pr);
    if (!ws) {
        ws_bytes = workspace_bytes(g);
        if ((st = ctx_workspace(ctx, ws_bytes, &ws)) != GF_OK) return st;
    }
    if (ws_bytes < workspace_bytes(g)) return fail(GF_ENOMEM, "workspace too small");
    if ((uintptr_t)ws % 256) return fail(GF_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    float *coef = (float *)ws;
    float *mean = coef + (size_t)(2 * g.C) * g.lps;
    float *lowres = mean + (size_t)(2 * g.C) * g.lps;
    const View vI{I->data, I->row_stride, I->plane_stride};
    const View vP{p->data, p->row_stride, p->plane_stride};
    // area subsampling: the low-res planes are made once; the candidates of
    // the coefficient kernel read them
    if (area_pass(g)) {
        const hipError_t e = launch_area(I->dtype, vI, vP, false, lowres, g, s);
        if (e != hipSuccess) return fail(GF_EDEVICE, "area subsampling launch failed: %s", hipGetErrorString(e));
    }

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(GF_EDEVICE, "hipEventCreate failed");
    }
    TileCfg chosen = default_tiles(g);
    // with the box means fused into the output pass, the box tile height
    // sets the fused pass's column runs: its candidates time that pass
    const View vQ{q->data, q->row_stride, q->plane_stride};
    const int mode = ctx->fuse.load();
    const bool fuse = (mode == GF_FUSE_ON || (mode == GF_FUSE_AUTO && fuse_pays(g))) &&
                      fused_px(g, chosen, I->dtype) > 0;
    int nres = 0;
    st = GF_OK;
    for (int kernel : {GF_K_COEFF, GF_K_BOX}) {
        double best_ms = 1e30;
        TileCfg best_cfg = chosen;
        for (const TileCfg &c : candidates(g, chosen, kernel)) {
            const int fpx = kernel == GF_K_BOX && fuse ? fused_px(g, c, I->dtype) : 0;
            if (kernel == GF_K_BOX && fuse && !fpx) continue;
            auto launch = [&]() -> hipError_t {
                if (fpx) return launch_outbox(I->dtype, vI, vQ, coef, g, c, fpx, s);
                if (kernel != GF_K_COEFF) return launch_box(coef, mean, g, c, s);
                return area_pass(g) ? launch_coeff_lowres(lowres, lowres + g.lps, coef, g, c, s)
                                    : launch_coeff(I->dtype, vI, vP, coef, g, c, s);
            };
            hipError_t e = launch();  // warm-up (also leaves valid a, b for the box candidates)
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int i = 0; e == hipSuccess && i < reps; ++i) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = fail(GF_EDEVICE, "tuning launch failed: %s", hipGetErrorString(e));
                break;
            }
            const double per = (double)ms / reps;
            if (results && nres < max_results)
                results[nres] = gf_tune_result{fpx ? GF_K_OUTPUT : kernel, to_abi(c), per};
            ++nres;
            if (per < best_ms) {
                best_ms = per;
                best_cfg = c;
            }
        }
        if (st != GF_OK) break;
        chosen = best_cfg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_results) *n_results = nres < max_results ? nres : max_results;
    if (st != GF_OK) return st;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        ctx->tuned[tile_key(I->dtype, I->h, I->w, p->c, pr->r, pr->s)] = chosen;
    }
    if (best) *best = to_abi(chosen);
    // leave q holding a valid result computed with the chosen shapes
    return run_fast(ctx, I, p, q, pr, ws, ws_bytes, s, &chosen);
}

gf_status gf_ctx_save_tuning(gf_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(GF_EINVAL, "gf_ctx_save_tuning: null argument");
    FILE *f = fopen(path, "w");
    if (!f) return fail(GF_EINVAL, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    // entries in key order, so the same choices always give the same file
    std::vector<std::pair<uint64_t, TileCfg>> entries(ctx->tuned.begin(), ctx->tuned.end());
    std::sort(entries.begin(), entries.end(),
              [](const std::pair<uint64_t, TileCfg> &a, const std::pair<uint64_t, TileCfg> &b) { return a.first < b.first; });
    fprintf(f, "{\"format\": \"gf-tiles-1\", \"arch\": \"gfx950\", \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : entries) {
        const TileCfg &t = kv.second;
        fprintf(f, "{\"key\": %llu, \"coeff_th\": %d, \"box_th\": %d}%s\n",
                (unsigned long long)kv.first, t.coeff_th, t.box_th, ++i < entries.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    return ok ? GF_OK : fail(GF_EINVAL, "write to %s failed", path);
}

gf_status gf_ctx_load_tuning(gf_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(GF_EINVAL, "gf_ctx_load_tuning: null argument");
    FILE *f = fopen(path, "r");
    if (!f) return fail(GF_EINVAL, "cannot open %s", path);
    char line[512];
    gf_status st = GF_OK;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, "\"key\"")) continue;
        unsigned long long key = 0;
        TileCfg t;
        if (sscanf(line, " {\"key\": %llu, \"coeff_th\": %d, \"box_th\": %d", &key, &t.coeff_th,
                   &t.box_th) != 3) {
            st = fail(GF_EINVAL, "malformed tuning entry in %s: %s", path, line);
            break;
        }
        ctx->tuned[(uint64_t)key] = t;
    }
    fclose(f);
    return st;
}

gf_status gf_tune_batched(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p, gf_image *q,
                          const gf_params *pr, void *ws, size_t ws_bytes, void *stream, int32_t reps,
                          gf_batch_cfg *best, gf_batch_tune_result *results, int32_t max_results,
                          int32_t *n_results) {
    if (!ctx) return fail(GF_EINVAL, "gf_tune_batched needs a context");
    if (n_results) *n_results = 0;
    if (reps < 1) reps = 5;
    gf_status st;
    if ((st = ctx_use_device(ctx)) != GF_OK) return st;
    const gf_batch_cfg saved = ctx_batch_cfg(ctx);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(GF_EDEVICE, "hipEventCreate failed");
    }
    gf_batch_cfg win{};
    double win_ms = 0.0;
    int found = 0, nres = 0;
    st = GF_OK;
    // The phase schedule's tile heights are the candidates.  The queue
    // schedule (one persistent kernel holding every phase's LDS and
    // registers, so two or three workgroups per CU) is a candidate only when
    // the context is set to it: on the 256-image mix it took 6.7 ms against
    // 1.9 ms for the phase grids.
    const bool queue = saved.schedule == GF_BATCH_QUEUE;
    for (int sched : {GF_BATCH_PHASES, GF_BATCH_QUEUE}) {
        if ((sched == GF_BATCH_QUEUE) != queue) continue;
        for (int th : {8, 16, 24, 32, 48}) {
            const gf_batch_cfg c{sched, th};
            BatchPlan plan;
            if ((st = plan_batch(n, I, p, q, pr, (char *)ws, c, &plan)) != GF_OK) break;
            if (plan.th != th) continue;  // does not fit at this batch's largest radius
            (void)gf_ctx_set_batch_cfg(ctx, &c);
            if ((st = gf_fast_batched(ctx, n, I, p, q, pr, ws, ws_bytes, stream)) != GF_OK) break;
            hipError_t e = hipEventRecord(e0, s);
            for (int k = 0; k < reps && st == GF_OK; ++k) st = gf_fast_batched(ctx, n, I, p, q, pr, ws, ws_bytes, stream);
            if (st != GF_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = fail(GF_EDEVICE, "timing: %s", hipGetErrorString(e));
                break;
            }
            const double per = (double)ms / reps;
            if (results && nres < max_results) results[nres++] = gf_batch_tune_result{c, per};
            if (!found || per < win_ms) {
                win = c;
                win_ms = per;
                found = 1;
            }
        }
        if (st != GF_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_results) *n_results = nres;
    if (st != GF_OK || !found) {
        (void)gf_ctx_set_batch_cfg(ctx, &saved);
        return st != GF_OK ? st : fail(GF_ENOTSUP, "no batched configuration fits this batch");
    }
    (void)gf_ctx_set_batch_cfg(ctx, &win);
    if (best) *best = win;
    if ((st = gf_fast_batched(ctx, n, I, p, q, pr, ws, ws_bytes, stream)) != GF_OK) return st;
    const hipError_t e = hipStreamSynchronize(s);
    return e == hipSuccess ? GF_OK : fail(GF_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
}

}  // extern "C"
