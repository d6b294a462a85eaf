// Internal declarations shared by the host API (gf_api.cpp) and the HIP
// kernels (gf_kernels.hip, gf_batched.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "gf.h"

namespace gf {

// Geometry of one filtering problem.  Full-res H x W, low-res Hl x Wl
// (ceil(H/s) x ceil(W/s)), low-res radius R, G channels of the guide (1
// gray, 3 colour), C channels of p, subsampling kind sub and border
// convention border (gf_subsample, gf_border).  The
// low-resolution FP32 maps live in a workspace as planes of Hl rows with
// row stride lrs (a multiple of 16 floats) and plane stride lps (a multiple
// of 64 floats), so every plane and row start is 64-byte aligned.
// refl_h, refl_w: reflections a reflect-101 border needs on each axis to
// bring every position a window reaches back into the map (1 unless the
// window is wider than the map; 0 for the other borders).
struct Geo {
    int H, W;
    int Hl, Wl;
    int s, R, G, C, sub, border;
    int refl_h, refl_w;
    float eps;
    int64_t lrs, lps;
};

// Strided view of a device image: element (k, y, x) at data + k*ps + y*rs + x.
struct View {
    void *data;
    int64_t rs, ps;
};

// Tile shapes for one call (picked by the host heuristic or the tuner).
struct TileCfg {
    int coeff_th;  // rows of a coefficient tile (8, 16, 24, 32, 48 or 64); tiles are 64 columns wide
    int box_th;    // rows of a box-mean tile (8, 16, 24, 32, 48 or 64)
};

constexpr int kThreads = 256;   // threads per workgroup for every kernel
constexpr int kTileW = 64;      // low-res tile width of the window-sum kernels
constexpr int kRun = 8;         // consecutive outputs per thread in a row pass
constexpr int kOutPx = 4;       // full-res pixels per lane in the output kernel
constexpr int kOutTileW = 64 * kOutPx;  // full-res columns per output tile
// Dynamic LDS that every output-pass launch reserves and never touches: with
// it at most three workgroups (12 waves) share a CU.  The pass writes HBM
// faster with fewer waves in flight than its registers allow (four or more):
// on the 4000x3000 RGB fp32 output pass 37.4 -> 35.3 us at s = 4, 36.2 ->
// 32.6 at s = 8, 45.1 -> 41.5 at s = 2, 97.5 -> 87.8 at s = 1.  Kernels that
// their registers already hold to three workgroups per CU are unaffected.
constexpr size_t kOutResidencyLds = 48 << 10;
constexpr int kMaxRadius = 64;  // largest low-res radius the LDS tile buffers hold
constexpr int kCUs = 256;       // compute units of an MI355X (grid-size heuristics)
// Polls of the queue schedule's bounded wait before a tile gives up on the
// previous phase of its image (about three seconds); gf_ctx_set_wait_limit.
constexpr unsigned kBatchSpinLimit = 1u << 26;

Geo make_geo(int H, int W, int C, const gf_params &pr, int G = 1);
// Area subsampling runs as a pass of its own (launch_area) into FP32 planes.
inline bool area_pass(const Geo &g) { return g.sub == GF_SUB_AREA && g.s > 1; }
constexpr size_t kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950

// LDS layout of the window-sum tiles (gf_device.h, gf_color.h), needed by
// the host to pick tile heights: row-sum planes of kRowW elements per row,
// staged regions of region_stride(R) floats per row (odd, so that lanes on
// consecutive rows fall in different banks).  constexpr functions serve
// host and device code alike.
constexpr int kRowW = 65;
constexpr int region_stride(int R) { return (kTileW + 2 * R) | 1; }
// coefficient tile: two FP64 row-sum planes, and with `stage` the guide's
// and one channel's samples
constexpr size_t coeff_tile_lds(int TH, int R, bool stage) {
    return (size_t)2 * (TH + 2 * R) * kRowW * sizeof(double) +
           (stage ? (size_t)2 * (TH + 2 * R) * region_stride(R) * sizeof(float) : 0);
}
// box-mean tile: one FP32 row-sum plane and the staged map region
constexpr size_t box_tile_lds(int TH, int R) {
    return (size_t)(TH + 2 * R) * kRowW * sizeof(float) + (size_t)(TH + 2 * R) * region_stride(R) * sizeof(float);
}
// colour coefficient tile: two FP64 row-sum planes and four staged regions
// (the guide's three channels and one channel of p)
constexpr size_t color_tile_lds(int TH, int R) {
    return (size_t)2 * (TH + 2 * R) * kRowW * sizeof(double) +
           (size_t)4 * (TH + 2 * R) * region_stride(R) * sizeof(float);
}
// Box means fused into the output pass (gf_outbox.h): a block of q is
// kObRows full-res rows by 64 PX columns.  Low-res rows (columns) that n
// consecutive full-res rows (columns) at ratio s >= 2 interpolate from: at
// most ceil((n - 1) / s) + 2; runs of length L starting at multiples of L
// that cover any np consecutive positions: at most ceil((np - 1) / L) + 1.
constexpr int kObRows = 32;
constexpr int ob_patch(int n, int s) { return (n - 1 + s - 1) / s + 2; }
constexpr int ob_runs(int np, int L) { return (np - 1 + L - 1) / L + 1; }
constexpr int ob_rows_max(int s, int LC) { return LC * ob_runs(ob_patch(kObRows, s), LC); }
constexpr int ob_cols_max(int s, int PX) { return kRun * ob_runs(ob_patch(64 * PX, s), kRun); }
// LDS of a fused block: row sums of a and b over the computed columns for
// every region row (computed rows + 2R), then the patches of mean_a and
// mean_b; rows of (computed columns + 1) floats.
constexpr size_t outbox_lds(int s, int R, int LC, int PX) {
    return sizeof(float) * (size_t)(ob_cols_max(s, PX) + 1) *
           (size_t)(2 * (ob_rows_max(s, LC) + 2 * R) + 2 * ob_rows_max(s, LC));
}
bool coeff_staged(const TileCfg &t, int R);
size_t coeff_lds_bytes(const TileCfg &t, int R);
size_t box_lds_bytes(const TileCfg &t, int R);
TileCfg default_tiles(const Geo &g);

// Timing events of one launcher call (null: none).  The launcher passes them
// to the dispatch itself (hipExtLaunchKernel), start with its first kernel
// and stop with its last, so they time the kernels and nothing between.
struct Stamp {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Output epilogue: detail enhancement e = q + gain (p - q), p full resolution
// with the layout of q (data null: plain q).
struct Detail {
    View p{};
    float gain = 0.f;
};

// Kernel launchers (gf_kernels.hip).  All return the launch status.
// p_low: p is given at low resolution (joint upsampling) and read as is.
hipError_t launch_coeff(gf_dtype dt, const View &I, const View &P, float *coef,
                        const Geo &g, const TileCfg &t, hipStream_t st, const Stamp &ts = Stamp{},
                        bool p_low = false);
hipError_t launch_box(const float *src, float *dst, const Geo &g, const TileCfg &t,
                      hipStream_t st, const Stamp &ts = Stamp{});
// Area subsampling of the G channels of I (planes 0..G-1 of dst) and of the
// C channels of P (planes G..G+C-1; with p_low, P is already low-res and is
// converted as it is), FP32 planes of stride g.lps.  The coefficients then
// come from launch_coeff_lowres (or its colour form).
hipError_t launch_area(gf_dtype dt, const View &I, const View &P, bool p_low, float *dst, const Geo &g,
                       hipStream_t st, const Stamp &ts = Stamp{});
// Coefficients from low-res FP32 planes: guide Il, channels of p at Pl + c*g.lps.
hipError_t launch_coeff_lowres(const float *Il, const float *Pl, float *coef, const Geo &g, const TileCfg &t,
                               hipStream_t st, const Stamp &ts = Stamp{});
// The same launchers for the padded borders (gf_kernels_padded.hip); the
// launchers above forward to them when g.border is not GF_BORDER_CLIP.
hipError_t launch_coeff_padded(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g,
                               const TileCfg &t, hipStream_t st, const Stamp &ts, bool p_low);
hipError_t launch_coeff_lowres_padded(const float *Il, const float *Pl, float *coef, const Geo &g,
                                      const TileCfg &t, hipStream_t st, const Stamp &ts);
hipError_t launch_box_padded(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st,
                             const Stamp &ts);
hipError_t launch_output(gf_dtype dt, const View &I, const View &Q, const float *mean,
                         const Geo &g, const TileCfg &t, hipStream_t st,
                         const Stamp &ts = Stamp{}, const Detail &detail = Detail{});

// Box means fused into the output pass (gf_kernels_outbox.hip), for a gray
// guide at s in {2, 4, 8}: fused_px gives the pixels per lane of the fused
// launch for this problem, tiles (the box tile height sets its column runs)
// and dtype, or 0 when the fused pass does not apply (other ratios, a colour
// guide, LDS above kObLdsMax).  launch_outbox then replaces launch_box +
// launch_output, reading a, b (coef: 2C planes) and writing q with the same
// bits.
// fuse_pays: the built-in choice (GF_FUSE_AUTO) takes the fused pass for
// one channel of p on low-res maps of at most kFuseMaxLowres pixels, where
// the launches are latency-bound and one fewer pays (a 512x512 image at
// s = 4: 17.5 us against 20.9); with more channels, or on larger maps, the
// fused pass's halo work and its serial channel loop cost more than the
// separate pass (512x512 RGB: 28.1 us against 22.0).
constexpr size_t kObLdsMax = 80 * 1024;
constexpr int64_t kFuseMaxLowres = 1 << 16;
int fused_px(const Geo &g, const TileCfg &t, gf_dtype dt);
bool fuse_pays(const Geo &g);
hipError_t launch_outbox(gf_dtype dt, const View &I, const View &Q, const float *coef, const Geo &g,
                         const TileCfg &t, int px, hipStream_t st, const Stamp &ts = Stamp{},
                         const Detail &detail = Detail{});

// Colour guide (gf_kernels_color.hip): coefficients a_0..a_2, b per channel
// (4C planes at coef, layout in gf_color.h), from the images or from the
// low-res FP32 planes of area subsampling (guide Il: 3 planes; p: Pl + c*lps;
// p_low: p given at low resolution, joint upsampling); output q (or, with a
// detail epilogue, e) from the box means of those 4C planes.
// color_tile_h: the coefficient tile height used for tiles t at radius R
// (16 where it fits unless t pins fewer rows, else 8; 0 when even 8 rows
// do not fit in LDS).
int color_tile_h(const TileCfg &t, int R);
hipError_t launch_coeff_color(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                              hipStream_t st, const Stamp &ts = Stamp{}, bool p_low = false);
hipError_t launch_coeff_color_lowres(const float *Il, const float *Pl, float *coef, const Geo &g, const TileCfg &t,
                                     hipStream_t st, const Stamp &ts = Stamp{});
hipError_t launch_output_color(gf_dtype dt, const View &I, const View &Q, const float *mean, const Geo &g,
                               hipStream_t st, const Stamp &ts = Stamp{}, const Detail &detail = Detail{});

}  // namespace gf
