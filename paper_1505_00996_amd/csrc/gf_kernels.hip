// Per-image kernels of the (fast) guided filter for gfx950 and their host
// launchers.  Algorithm 2 of He & Sun, "Fast Guided Filter", runs as three
// launches on the caller's stream:
//   k_coeff  (grid: low-res tiles)             steps 1-4 -> a, b (all channels)
//   k_box    (grid: low-res tiles x 2C maps)   step 5    -> mean_a, mean_b
//   k_output (grid: full-res (4 x 64 PX) x 8 blocks) steps 6-7 -> q
// Algorithm 1 is the same three launches at s = 1, where subsampling and
// upsampling are identities.  Area subsampling adds a first launch,
//   k_area   (grid: low-res 256 x 1 blocks x (G+C) planes)  step 1 -> I', p'
// after which k_coeff reads the FP32 low-res planes as they are.  The
// per-tile work lives in gf_device.h; the window-sum kernels and their
// launchers in gf_window_kernels.h (this file instantiates the
// clip-normalised ones, gf_kernels_padded.hip the padded-border ones).
#include "gf_window_kernels.h"

namespace gf {
namespace {

// Pixels per lane of the per-image output kernel: every row access is 16
// bytes (4 fp32 or 8 16-bit values).
template <typename T>
constexpr int out_px() { return sizeof(T) == 2 ? 8 : 4; }

// One workgroup = 4 waves side by side = a (4 x 64 PX)-column x 8-row block
// of q (EPI: of the detail-enhanced e, reading the matching block of p).
template <typename T, int CC, int S, bool EPI>
__global__ __launch_bounds__(kThreads) void k_output(const T *__restrict__ I, int64_t Irs,
                                                     T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                     const float *__restrict__ M, Geo g, int c0,
                                                     int ntx, int ntiles, const T *__restrict__ P,
                                                     int64_t Prs, int64_t Pps, float gain) {
    constexpr int PX = out_px<T>();
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    output_rows<T, CC, S, EPI, PX>(I, Irs, Q, Qrs, Qps, M, g, c0, (tile / ntx) * kOutRows,
                                   ((tile % ntx) * 4 + wave_id()) * (64 * PX), P, Prs, Pps, gain);
}

// Area subsampling (step 1 with the block mean): low-res pixel (ly, lx) of
// plane k is the mean of the full-res block [s*ly, s*ly+s) x [s*lx, s*lx+s)
// clipped to the image, summed in FP64 row by row and rounded once to FP32.
// Planes 0..G-1 are the guide's channels (1 gray, 3 colour), planes
// G..G+C-1 the channels of p; with p_low those are given at low resolution
// and are converted as they are.  A workgroup covers one low-res row x 256
// columns (its four waves side by side, one column per lane) of plane
// blockIdx.y.  S: compile-time ratio for full blocks (0: g.s at run time);
// every row of a full block is read with 2- or 4-wide loads (one
// instruction at any element-aligned address).
template <typename T, int S>
__global__ __launch_bounds__(kThreads) void k_area(const T *__restrict__ I, int64_t Irs, int64_t Ips,
                                                   const T *__restrict__ P, int64_t Prs, int64_t Pps, int p_low,
                                                   float *__restrict__ dst, Geo g, int ntx) {
    const int lane = threadIdx.x & 63;
    const int ly = blockIdx.x / ntx, lx = ((blockIdx.x % ntx) * 4 + wave_id()) * 64 + lane;
    if (ly >= g.Hl || lx >= g.Wl) return;  // no barriers in this kernel
    const int k = blockIdx.y;
    float *out = dst + (int64_t)k * g.lps + (int64_t)ly * g.lrs + lx;
    if (k >= g.G && p_low) {
        *out = ld(P + (int64_t)(k - g.G) * Pps + (int64_t)ly * Prs + lx);
        return;
    }
    const T *src = k < g.G ? I + (int64_t)k * Ips : P + (int64_t)(k - g.G) * Pps;
    const int64_t rs = k < g.G ? Irs : Prs;
    const int s = S ? S : g.s, y0 = s * ly, x0 = s * lx;
    const int ny = min(s, g.H - y0), nx = min(s, g.W - x0);  // >= 1: s*ly < H, s*lx < W
    double acc = 0.0;
    if (S && ny == S && nx == S) {
        double ra[S > 0 ? S : 1];
        {
            // all loads first, then the sums (in the same order as the
            // ragged-block loop below)
            float v[S > 0 ? S : 1][S > 0 ? S : 1];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const T *row = src + (int64_t)(y0 + i) * rs + x0;
                if constexpr (S == 2) {
                    const f32x2 a = ld2(row);
                    v[i][0] = a[0];
                    v[i][1] = a[1];
                } else {
#pragma unroll
                    for (int j = 0; j < S; j += 4) {
                        const f32x4 a = ld4(row + j);
                        v[i][j] = a[0];
                        v[i][j + 1] = a[1];
                        v[i][j + 2] = a[2];
                        v[i][j + 3] = a[3];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < S; ++i) {
                ra[i] = 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) ra[i] += (double)v[i][j];
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) acc += ra[i];
    } else {
        for (int i = 0; i < ny; ++i) {
            const T *row = src + (int64_t)(y0 + i) * rs + x0;
            double ra = 0.0;
            for (int j = 0; j < nx; ++j) ra += (double)ld(row + j);
            acc += ra;
        }
    }
    *out = (float)(acc / (double)(ny * nx));
}

template <typename T>
hipError_t area_t(const View &I, const View &P, bool p_low, float *dst, const Geo &g, hipStream_t st,
                  const Stamp &ts) {
    const int ntx = (g.Wl + 255) / 256, nty = g.Hl;
    const dim3 grid(ntx * nty, g.G + g.C), block(kThreads);
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
#define GF_AREA(SS)                                                                                  \
    launch_k(k_area<T, SS>, grid, block, 0, st, ts.start, ts.stop, Ip, I.rs, I.ps, Pp, P.rs, P.ps, (int)p_low, dst, \
             g, ntx)
    switch (g.s) {
        case 2: GF_AREA(2); break;
        case 4: GF_AREA(4); break;
        case 8: GF_AREA(8); break;
        default: GF_AREA(0); break;
    }
#undef GF_AREA
    return hipGetLastError();
}

template <typename T, int CC, bool EPI>
hipError_t output_cc(const View &I, const View &Q, const float *mean, const Geo &g, int c0, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const Detail &dt) {
    const int tw = 4 * 64 * out_px<T>();
    const int ntx = (g.W + tw - 1) / tw;
    const int nty = (g.H + kOutRows - 1) / kOutRows;
    const int ntiles = ntx * nty;
    const T *Ip = (const T *)I.data;
    T *Qp = (T *)Q.data + (int64_t)c0 * Q.ps;
    const T *Pp = EPI ? (const T *)dt.p.data + (int64_t)c0 * dt.p.ps : nullptr;
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_OUT(SS)                                                                                       \
    launch_k(k_output<T, CC, SS, EPI>, grid, block, kOutResidencyLds, st, e0, e1, Ip, I.rs, Qp, Q.rs, Q.ps, mean, g, c0, ntx, \
             ntiles, Pp, dt.p.rs, dt.p.ps, dt.gain)
    switch (g.s) {
        case 1: GF_OUT(1); break;
        case 2: GF_OUT(2); break;
        case 4: GF_OUT(4); break;
        case 8: GF_OUT(8); break;
        default: GF_OUT(0); break;
    }
#undef GF_OUT
    return hipGetLastError();
}

template <typename T, bool EPI>
hipError_t output_te(const View &I, const View &Q, const float *mean, const Geo &g, hipStream_t st, const Stamp &ts, const Detail &dt) {
    for (int c0 = 0; c0 < g.C; c0 += 3) {
        const int cc = g.C - c0 < 3 ? g.C - c0 : 3;
        const hipEvent_t e0 = c0 == 0 ? ts.start : nullptr, e1 = c0 + 3 >= g.C ? ts.stop : nullptr;
        hipError_t e = cc == 3 ? output_cc<T, 3, EPI>(I, Q, mean, g, c0, st, e0, e1, dt)
                     : cc == 2 ? output_cc<T, 2, EPI>(I, Q, mean, g, c0, st, e0, e1, dt)
                               : output_cc<T, 1, EPI>(I, Q, mean, g, c0, st, e0, e1, dt);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t output_t(const View &I, const View &Q, const float *mean, const Geo &g, hipStream_t st,
                    const Stamp &ts, const Detail &dt) {
    return dt.p.data ? output_te<T, true>(I, Q, mean, g, st, ts, dt) : output_te<T, false>(I, Q, mean, g, st, ts, dt);
}

}  // namespace

hipError_t launch_coeff(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g,
                        const TileCfg &t, hipStream_t st, const Stamp &ts, bool p_low) {
    if (g.border != GF_BORDER_CLIP) return launch_coeff_padded(dt, I, P, coef, g, t, st, ts, p_low);
    return coeff_dt<kClip>(dt, I, P, coef, g, t, st, ts, p_low);
}

hipError_t launch_area(gf_dtype dt, const View &I, const View &P, bool p_low, float *dst, const Geo &g,
                       hipStream_t st, const Stamp &ts) {
    switch (dt) {
        case GF_F32: return area_t<float>(I, P, p_low, dst, g, st, ts);
        case GF_F16: return area_t<_Float16>(I, P, p_low, dst, g, st, ts);
        case GF_BF16: return area_t<dev::bf16>(I, P, p_low, dst, g, st, ts);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_coeff_lowres(const float *Il, const float *Pl, float *coef, const Geo &g, const TileCfg &t,
                               hipStream_t st, const Stamp &ts) {
    if (g.border != GF_BORDER_CLIP) return launch_coeff_lowres_padded(Il, Pl, coef, g, t, st, ts);
    return coeff_lowres<kClip>(Il, Pl, coef, g, t, st, ts);
}

hipError_t launch_box(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st,
                      const Stamp &ts) {
    if (g.border != GF_BORDER_CLIP) return launch_box_padded(src, dst, g, t, st, ts);
    return box_b<kClip>(src, dst, g, t, st, ts);
}

hipError_t launch_output(gf_dtype dt, const View &I, const View &Q, const float *mean, const Geo &g,
                         const TileCfg &, hipStream_t st, const Stamp &ts, const Detail &detail) {
    switch (dt) {
        case GF_F32: return output_t<float>(I, Q, mean, g, st, ts, detail);
        case GF_F16: return output_t<_Float16>(I, Q, mean, g, st, ts, detail);
        case GF_BF16: return output_t<dev::bf16>(I, Q, mean, g, st, ts, detail);
    }
    return hipErrorInvalidValue;
}

}  // namespace gf
