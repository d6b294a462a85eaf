// Host side of libgf.so: argument validation, geometry, workspace layout,
// tile heuristics and the gf_plain / gf_fast entry points of include/gf.h.
// Validation is pure host code and runs before any HIP call, so an invalid
// call is reported without touching a device.
#include <hip/hip_runtime_api.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "gf_api_internal.h"
#include "gf_internal.h"

namespace gf {

static thread_local char t_err[512] = "";

gf_status fail(gf_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof t_err, fmt, ap);
    va_end(ap);
    return st;
}

const char *last_error() { return t_err; }

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int lowres_radius(int r, int s) {
    if (r <= 0) return 0;
    const int rl = (2 * r + s) / (2 * s);  // r/s rounded half up
    return rl < 1 ? 1 : rl;
}

// Applications of the reflection F(m) = (n-1) - |(n-1) - |m|| that bring
// every position in [-R, n-1+R] into [0, n) (the device applies them in
// pad_index); 1 when the window is no wider than the axis allows.
static int reflections(int n, int R) {
    if (n <= 1) return 1;
    int most = 1;
    for (int i : {-R, n - 1 + R}) {
        int m = i, k = 0;
        do {
            m = n - 1 - std::abs(n - 1 - std::abs(m));
            ++k;
        } while (m < 0 || m > n - 1);
        most = std::max(most, k);
    }
    return most;
}

Geo make_geo(int H, int W, int C, const gf_params &pr, int G) {
    Geo g;
    g.G = G;
    const int s = pr.s;
    g.H = H;
    g.W = W;
    g.s = s;
    g.Hl = (H + s - 1) / s;
    g.Wl = (W + s - 1) / s;
    g.R = lowres_radius(pr.r, s);
    g.C = C;
    g.sub = (int)pr.sub;
    g.border = (int)pr.border;
    const bool refl = pr.border == GF_BORDER_REFLECT101;
    g.refl_h = refl ? reflections(g.Hl, g.R) : 0;
    g.refl_w = refl ? reflections(g.Wl, g.R) : 0;
    g.eps = (float)pr.eps;
    g.lrs = round_up(g.Wl, 16);
    g.lps = round_up((int64_t)g.Hl * g.lrs, 64);
    return g;
}

static const size_t kLdsMax = kLdsLimit;

// Staged coefficient tiles when they fit; otherwise unstaged 8-row tiles.
bool coeff_staged(const TileCfg &t, int R) { return coeff_tile_lds(t.coeff_th, R, true) <= kLdsLimit; }
size_t coeff_lds_bytes(const TileCfg &t, int R) {
    return coeff_staged(t, R) ? coeff_tile_lds(t.coeff_th, R, true) : coeff_tile_lds(8, R, false);
}
size_t box_lds_bytes(const TileCfg &t, int R) { return box_tile_lds(t.box_th, R); }

// 16-row tiles where they fit in LDS (6% faster than 8 rows at r' = 4, 38%
// at r' = 16, although at about 245 VGPRs two waves fit per SIMD against
// three at 8 rows), 8 rows when the tiles are pinned below 16 or 16 do not
// fit; 0 when none fits.
int color_tile_h(const TileCfg &t, int R) {
    if (t.coeff_th >= 16 && color_tile_lds(16, R) <= kLdsLimit) return 16;
    return color_tile_lds(8, R) <= kLdsLimit ? 8 : 0;
}

static bool th_ok(int th) { return th == 8 || th == 16 || th == 24 || th == 32 || th == 48 || th == 64; }

// Tile heights: tall tiles amortise the 2r' halo rows, short ones give the
// grid more workgroups.  The choices follow sweeps of both kernels (r' = 2..32
// on a 12 MP image; at r' <= 4 also maps of 128x128 to 1000x750).
// Coefficients at r' <= 4: 24 rows when that gives at least 192 tiles (the
// 4000x3000 map at s = 4: 22.2 us against 22.8 at 16 rows), else 16 when
// that gives at least 128, else 8 (a 128x128 map: 6.5 us against 8.1 at 24
// rows); up to r' = 10, 32 rows; then the tallest tile whose region still
// fits in LDS.  Box means at r' <= 4: 48 rows when the box grid keeps at
// least 1024 workgroups (the 4000x3000 RGB map at s = 4: 15.1 us against 16.0
// at 24 rows), else 24 when that gives at least 128, else 8 (a 128x128 map:
// 3.8 us against 4.5 at 24); up to r' = 16, 48 rows; then the tallest tile
// that leaves room for two workgroups per CU.
static int pick_coeff_th(const Geo &g) {
    const int R = g.R;
    auto fits = [&](int th) {
        const TileCfg t{th, th};
        return coeff_staged(t, R) && coeff_lds_bytes(t, R) <= kLdsMax;
    };
    auto tiles = [&](int th) { return (int64_t)((g.Wl + kTileW - 1) / kTileW) * ((g.Hl + th - 1) / th); };
    if (R <= 4 && fits(24)) return tiles(24) >= 192 ? 24 : tiles(16) >= 128 ? 16 : 8;
    if (R <= 10 && fits(32)) return 32;
    for (int th : {64, 48, 32, 24, 16})
        if (fits(th)) return th;
    return 8;  // unstaged 8-row tiles
}

static int pick_box_th(const Geo &g) {
    const int R = g.R;
    auto fits = [&](int th, size_t room) { return box_lds_bytes(TileCfg{th, th}, R) <= room; };
    // workgroups of the box grid: tiles of one plane times its 2C planes
    auto groups = [&](int th) { return (int64_t)((g.Wl + kTileW - 1) / kTileW) * ((g.Hl + th - 1) / th) * 2 * g.C; };
    if (R <= 4) {
        if (fits(48, kLdsMax) && groups(48) >= 1024) return 48;
        return groups(24) >= 128 ? 24 : 8;
    }
    if (R <= 16 && fits(48, kLdsMax)) return 48;
    for (size_t room : {(size_t)80 * 1024, kLdsMax})
        for (int th : {64, 48, 32, 24, 16})
            if (fits(th, room)) return th;
    return 8;
}

int fused_px(const Geo &g, const TileCfg &t, gf_dtype dt) {
    if (g.G != 1 || !(g.s == 2 || g.s == 4 || g.s == 8) || !th_ok(t.box_th)) return 0;
    const int LC = t.box_th / 4;
    // 16-bit rows: eight pixels per lane (16-byte accesses) while the block's
    // LDS leaves room for four workgroups per CU, else four
    if (dt != GF_F32 && outbox_lds(g.s, g.R, LC, 8) <= kLdsLimit / 4) return 8;
    return outbox_lds(g.s, g.R, LC, 4) <= kObLdsMax ? 4 : 0;
}

bool fuse_pays(const Geo &g) { return g.C == 1 && (int64_t)g.Hl * g.Wl <= kFuseMaxLowres; }

TileCfg default_tiles(const Geo &g) {
    TileCfg t;
    t.coeff_th = pick_coeff_th(g);
    // box means fused into the output pass: runs of two rows (8-row box
    // tiles), which compute the fewest rows past a block's patch
    const TileCfg fused{t.coeff_th, 8};
    t.box_th = fuse_pays(g) && fused_px(g, fused, GF_F32) ? 8 : pick_box_th(g);
    return t;
}

bool tiles_fit(const Geo &g, const TileCfg &t) {
    return th_ok(t.coeff_th) && th_ok(t.box_th) && coeff_lds_bytes(t, g.R) <= kLdsMax &&
           box_lds_bytes(t, g.R) <= kLdsMax;
}

size_t workspace_bytes(const Geo &g) {
    // a, b (2C planes, or 4C with a colour guide: a_0..a_2, b) and their box
    // means, FP32; with area subsampling also the G channels of I' and the C
    // channels of p'
    const int maps = (g.G == 3 ? 4 : 2) * g.C;
    return sizeof(float) * (size_t)(2 * maps + (area_pass(g) ? g.G + g.C : 0)) * (size_t)g.lps;
}

static size_t elem_size(gf_dtype d) { return d == GF_F32 ? 4 : 2; }

// Byte range [lo, hi) touched by an image view.
static void extent(const gf_image *im, uintptr_t *lo, uintptr_t *hi) {
    const size_t es = elem_size(im->dtype);
    *lo = (uintptr_t)im->data;
    const int64_t last = (int64_t)(im->c - 1) * im->plane_stride +
                         (int64_t)(im->h - 1) * im->row_stride + im->w;
    *hi = *lo + (uintptr_t)(last * (int64_t)es);
}

static bool overlaps(const gf_image *a, const gf_image *b) {
    uintptr_t a0, a1, b0, b1;
    extent(a, &a0, &a1);
    extent(b, &b0, &b1);
    return a0 < b1 && b0 < a1;
}

static gf_status check_image(const gf_image *im, const char *name) {
    if (!im) return fail(GF_EINVAL, "%s: null descriptor", name);
    if (!im->data) return fail(GF_EINVAL, "%s: null data pointer", name);
    if (im->dtype != GF_F32 && im->dtype != GF_F16 && im->dtype != GF_BF16)
        return fail(GF_EINVAL, "%s: unknown dtype %d", name, (int)im->dtype);
    if (im->c < 1 || im->h < 1 || im->w < 1)
        return fail(GF_EINVAL, "%s: empty or negative shape %dx%dx%d", name, im->c, im->h, im->w);
    if (im->row_stride < im->w)
        return fail(GF_EINVAL, "%s: row_stride %lld < w %d", name, (long long)im->row_stride, im->w);
    if (im->c > 1 && im->plane_stride < (int64_t)im->h * im->row_stride)
        return fail(GF_EINVAL, "%s: plane_stride %lld < h*row_stride", name,
                    (long long)im->plane_stride);
    if ((uintptr_t)im->data % elem_size(im->dtype))
        return fail(GF_EINVAL, "%s: data pointer not aligned to its element size", name);
    return GF_OK;
}

gf_status validate(const gf_image *I, const gf_image *p, const gf_image *q,
                   const gf_params *pr, bool p_low) {
    gf_status st;
    if ((st = check_image(I, "I")) != GF_OK) return st;
    if ((st = check_image(p, "p")) != GF_OK) return st;
    if ((st = check_image(q, "q")) != GF_OK) return st;
    if (!pr) return fail(GF_EINVAL, "params: null");
    if (I->c != 1 && I->c != 3) return fail(GF_ENOTSUP, "I: a guide has 1 (gray) or 3 (colour) channels, not %d", I->c);
    if (pr->s < 1) return fail(GF_EINVAL, "s = %d < 1", pr->s);
    // p is full resolution, or (joint upsampling) ceil(h/s) x ceil(w/s)
    const int ph = p_low ? (I->h + pr->s - 1) / pr->s : I->h, pw = p_low ? (I->w + pr->s - 1) / pr->s : I->w;
    if (p->h != ph || p->w != pw || q->h != I->h || q->w != I->w)
        return fail(GF_EINVAL, "shape mismatch: I %dx%d, p %dx%d (expected %dx%d), q %dx%d", I->h, I->w, p->h,
                    p->w, ph, pw, q->h, q->w);
    if (p->c != q->c) return fail(GF_EINVAL, "channel mismatch: p has %d, q has %d", p->c, q->c);
    if (p->dtype != I->dtype || q->dtype != I->dtype)
        return fail(GF_EINVAL, "dtype mismatch between I, p and q");
    if (overlaps(q, I) || overlaps(q, p)) return fail(GF_EINVAL, "q overlaps I or p");
    if (pr->r < 0) return fail(GF_EINVAL, "r = %d < 0", pr->r);
    if (pr->s < 1) return fail(GF_EINVAL, "s = %d < 1", pr->s);
    if (!(pr->eps > 0.0) || !isfinite(pr->eps) || !((float)pr->eps > 0.0f) ||
        !isfinite((float)pr->eps))
        return fail(GF_EINVAL, "eps = %g must be positive and finite (in FP32)", pr->eps);
    if (pr->border != GF_BORDER_CLIP && pr->border != GF_BORDER_REPLICATE && pr->border != GF_BORDER_REFLECT101)
        return fail(GF_EINVAL, "unknown border convention %d", (int)pr->border);
    if (pr->sub != GF_SUB_NEAREST && pr->sub != GF_SUB_BILINEAR && pr->sub != GF_SUB_AREA)
        return fail(GF_EINVAL, "unknown subsampling mode %d", (int)pr->sub);
    if (I->h > (1 << 24) || I->w > (1 << 24)) return fail(GF_ENOTSUP, "image side above 2^24");
    if (lowres_radius(pr->r, pr->s) > kMaxRadius)
        return fail(GF_ENOTSUP, "low-res radius %d above %d", lowres_radius(pr->r, pr->s), kMaxRadius);
    if (I->c == 3) {
        if (!color_tile_h(TileCfg{8, 8}, lowres_radius(pr->r, pr->s)))
            return fail(GF_ENOTSUP, "colour guide: low-res radius %d too large for the LDS tiles",
                        lowres_radius(pr->r, pr->s));
    }
    return GF_OK;
}

gf_status run_fast(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                   const gf_params *pr, void *ws, size_t ws_bytes, hipStream_t st,
                   const TileCfg *tiles, bool p_low, const float *gain) {
    const Geo g = make_geo(I->h, I->w, p->c, *pr, I->c);
    const int mode = ctx ? ctx->fuse.load() : GF_FUSE_AUTO;
    // pinned or tuned shapes that do not fit this radius fall back to the built-in choice
    TileCfg t = (tiles && tiles_fit(g, *tiles)) ? *tiles : default_tiles(g);
    // fusion asked for: the built-in box runs for the fused pass (two rows)
    if (!(tiles && tiles_fit(g, *tiles)) && mode == GF_FUSE_ON && g.G == 1 &&
        fused_px(g, TileCfg{t.coeff_th, 8}, I->dtype))
        t.box_th = 8;
    if (!tiles_fit(g, t)) return fail(GF_ENOTSUP, "tile shapes do not fit in LDS for r'=%d", g.R);
    const size_t need = workspace_bytes(g);
    if (!ws) return fail(GF_EINVAL, "no workspace");
    if (ws_bytes < need)
        return fail(GF_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % 256) return fail(GF_EINVAL, "workspace not 256-byte aligned");
    const bool color = g.G == 3;
    const int maps = (color ? 4 : 2) * g.C;
    float *coef = (float *)ws;
    float *mean = coef + (size_t)maps * g.lps;
    float *lowres = mean + (size_t)maps * g.lps;  // area subsampling: I' (G planes), then p'
    const View vI{I->data, I->row_stride, I->plane_stride};
    const View vP{p->data, p->row_stride, p->plane_stride};
    const View vQ{q->data, q->row_stride, q->plane_stride};
    hipError_t e = hipSuccess;
    if (area_pass(g)) {
        ProfScope ps(ctx, GF_K_AREA, st, true);
        e = launch_area(I->dtype, vI, vP, p_low, lowres, g, st, ps.stamp());
        ps.commit(e == hipSuccess);
    }
    if (e == hipSuccess) {
        ProfScope ps(ctx, GF_K_COEFF, st, true);
        const float *pl = lowres + (size_t)g.G * g.lps;
        if (color)
            e = area_pass(g) ? launch_coeff_color_lowres(lowres, pl, coef, g, t, st, ps.stamp())
                             : launch_coeff_color(I->dtype, vI, vP, coef, g, t, st, ps.stamp(), p_low);
        else
            e = area_pass(g) ? launch_coeff_lowres(lowres, pl, coef, g, t, st, ps.stamp())
                             : launch_coeff(I->dtype, vI, vP, coef, g, t, st, ps.stamp(), p_low);
        ps.commit(e == hipSuccess);
    }
    const int fpx = !color && (mode == GF_FUSE_ON || (mode == GF_FUSE_AUTO && fuse_pays(g)))
                        ? fused_px(g, t, I->dtype) : 0;
    if (e == hipSuccess && fpx) {
        // box means fused into the output pass
        ProfScope ps(ctx, GF_K_OUTPUT, st, true);
        Detail dt;
        if (gain) {
            dt.p = vP;
            dt.gain = *gain;
        }
        e = launch_outbox(I->dtype, vI, vQ, coef, g, t, fpx, st, ps.stamp(), dt);
        ps.commit(e == hipSuccess);
        if (e != hipSuccess) return fail(GF_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        return GF_OK;
    }
    if (e == hipSuccess) {
        // the box tiles run over maps = 2 * gb.C planes
        Geo gb = g;
        gb.C = maps / 2;
        ProfScope ps(ctx, GF_K_BOX, st, true);
        e = launch_box(coef, mean, gb, t, st, ps.stamp());
        ps.commit(e == hipSuccess);
    }
    if (e == hipSuccess && color) {
        ProfScope ps(ctx, GF_K_OUTPUT, st, true);
        Detail dt;
        if (gain) {
            dt.p = vP;
            dt.gain = *gain;
        }
        e = launch_output_color(I->dtype, vI, vQ, mean, g, st, ps.stamp(), dt);
        ps.commit(e == hipSuccess);
    } else if (e == hipSuccess) {
        ProfScope ps(ctx, GF_K_OUTPUT, st, true);
        Detail dt;
        if (gain) {
            dt.p = vP;
            dt.gain = *gain;
        }
        e = launch_output(I->dtype, vI, vQ, mean, g, t, st, ps.stamp(), dt);
        ps.commit(e == hipSuccess);
    }
    if (e != hipSuccess) return fail(GF_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return GF_OK;
}

// Context-owned workspace, grown on demand.  Growing frees the old buffer
// after the device has finished with it.
gf_status ctx_workspace(gf_ctx *ctx, size_t need, void **ws) {
    if (ctx->ws_bytes < need) {
        if (ctx->ws) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return fail(GF_EDEVICE, "hipDeviceSynchronize: %s", hipGetErrorString(e));
            (void)hipFree(ctx->ws);
            ctx->ws = nullptr;
            ctx->ws_bytes = 0;
        }
        hipError_t e = hipMalloc(&ctx->ws, need);
        if (e != hipSuccess) {
            ctx->ws = nullptr;
            return fail(GF_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        ctx->ws_bytes = need;
    }
    *ws = ctx->ws;
    return GF_OK;
}

}  // namespace gf

using namespace gf;

extern "C" {

const char *gf_last_error(const gf_ctx *) { return gf::last_error(); }

size_t gf_workspace_bytes(int32_t h, int32_t w, int32_t c, const gf_params *pr) {
    return gf_workspace_bytes_guide(h, w, 1, c, pr);
}

size_t gf_workspace_bytes_guide(int32_t h, int32_t w, int32_t guide_c, int32_t c, const gf_params *pr) {
    if (!pr || h < 1 || w < 1 || c < 1 || pr->s < 1 || pr->r < 0 || (guide_c != 1 && guide_c != 3)) return 0;
    return workspace_bytes(make_geo(h, w, c, *pr, guide_c));
}

static gf_status fast_entry(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q, const gf_params *pr,
                            void *ws, size_t ws_bytes, void *stream, bool p_low, const float *gain = nullptr) {
    gf_status st = validate(I, p, q, pr, p_low);
    if (st != GF_OK) return st;
    if (!ws) {
        if (!ctx) return fail(GF_EINVAL, "workspace is NULL and there is no context");
        const Geo g = make_geo(I->h, I->w, p->c, *pr, I->c);
        if ((st = ctx_use_device(ctx)) != GF_OK) return st;
        ws_bytes = workspace_bytes(g);
        if ((st = ctx_workspace(ctx, ws_bytes, &ws)) != GF_OK) return st;
    } else if (ctx && (st = ctx_use_device(ctx)) != GF_OK) {
        return st;
    }
    TileCfg tuned;
    const bool have = ctx && ctx_tiles(ctx, I, p, pr, &tuned);
    return run_fast(ctx, I, p, q, pr, ws, ws_bytes, (hipStream_t)stream, have ? &tuned : nullptr, p_low, gain);
}

gf_status gf_fast(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                  const gf_params *pr, void *ws, size_t ws_bytes, void *stream) {
    return fast_entry(ctx, I, p, q, pr, ws, ws_bytes, stream, false);
}

gf_status gf_joint_upsample(gf_ctx *ctx, const gf_image *I, const gf_image *p_low, gf_image *q,
                            const gf_params *pr, void *ws, size_t ws_bytes, void *stream) {
    return fast_entry(ctx, I, p_low, q, pr, ws, ws_bytes, stream, true);
}

gf_status gf_detail_enhance(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *e,
                            const gf_params *pr, double gain, void *ws, size_t ws_bytes, void *stream) {
    const float g = (float)gain;
    if (!isfinite(gain) || !isfinite(g)) return fail(GF_EINVAL, "gain = %g must be finite (in FP32)", gain);
    return fast_entry(ctx, I, p, e, pr, ws, ws_bytes, stream, false, &g);
}

gf_status gf_plain(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q, int32_t r,
                   double eps, gf_border border, void *ws, size_t ws_bytes, void *stream) {
    gf_params pr;
    pr.r = r;
    pr.s = 1;
    pr.eps = eps;
    pr.border = border;
    pr.sub = GF_SUB_NEAREST;
    return gf_fast(ctx, I, p, q, &pr, ws, ws_bytes, stream);
}

}  // extern "C"
