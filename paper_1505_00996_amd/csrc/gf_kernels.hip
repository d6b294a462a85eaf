// Per-image kernels of the (fast) guided filter for gfx950 and their host
// launchers.  Algorithm 2 of He & Sun, "Fast Guided Filter", runs as three
// launches on the caller's stream:
//   k_coeff  (grid: low-res tiles)             steps 1-4 -> a, b (all channels)
//   k_box    (grid: low-res tiles x 2C maps)   step 5    -> mean_a, mean_b
//   k_output (grid: full-res 256 x 32 blocks)  steps 6-7 -> q
// Algorithm 1 is the same three launches at s = 1, where subsampling and
// upsampling are identities.  The per-tile work lives in gf_device.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "gf_device.h"
#include "gf_internal.h"

namespace gf {
namespace {

using namespace dev;

template <typename T, int K, int KP, int TH, bool STAGE>
__global__ __launch_bounds__(kThreads) void k_coeff(const T *__restrict__ I, int64_t Irs,
                                                    const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                                    float *__restrict__ coef, Geo g, int ntx, int ntiles) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    coeff_tile<T, K, TH, STAGE, false, KP>(I, Irs, P, Prs, Pps, coef, g, (tile / ntx) * TH, (tile % ntx) * kTileW,
                                           lds_d);
}

template <int TH>
__global__ __launch_bounds__(kThreads) void k_box(const float *__restrict__ src, float *__restrict__ dst,
                                                  Geo g, int ntx, int ntiles) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    box_tile<TH>(src + (int64_t)blockIdx.y * g.lps, dst + (int64_t)blockIdx.y * g.lps, g,
                 (tile / ntx) * TH, (tile % ntx) * kTileW, lds_d);
}

// One workgroup = 4 waves = a 256-column x 32-row block of q (EPI: of the
// detail-enhanced e, reading the matching block of p).
template <typename T, int CC, int S, bool EPI>
__global__ __launch_bounds__(kThreads) void k_output(const T *__restrict__ I, int64_t Irs,
                                                     T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                     const float *__restrict__ M, Geo g, int c0,
                                                     int ntx, int ntiles, int vec, const T *__restrict__ P,
                                                     int64_t Prs, int64_t Pps, float gain) {
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    output_rows<T, CC, S, EPI>(I, Irs, Q, Qrs, Qps, M, g, c0,
                               (tile / ntx) * (4 * kOutRows) + wave_id() * kOutRows,
                               (tile % ntx) * kOutTileW, vec != 0, P, Prs, Pps, gain);
}

int grid8(int n) { return ((n + 7) / 8) * 8; }

// A launch that carries timing events in its dispatch when asked to.
template <typename Kn, typename... A>
void launch_k(Kn kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
              A... args) {
    if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, e0, e1, 0u, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

// Dynamic LDS above 64 KB has to be allowed per kernel (gfx950 has 160 KB).
template <typename Kn>
void allow_lds(Kn kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

template <typename T, int K, int KP>
hipError_t coeff_tk(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                    hipStream_t st, const Stamp &ts) {
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
    const bool staged = coeff_staged(t, g.R);
    const int th = staged ? t.coeff_th : 8;  // the unstaged kernel works on 8-row tiles
    const int ntx = (g.Wl + kTileW - 1) / kTileW, nty = (g.Hl + th - 1) / th;
    const int ntiles = ntx * nty;
    const size_t lds = coeff_lds_bytes(t, g.R);
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_COEFF(TH, STG)                                                                              \
    {                                                                                                   \
        allow_lds(k_coeff<T, K, KP, TH, STG>, lds);                                                     \
        launch_k(k_coeff<T, K, KP, TH, STG>, grid, block, lds, st, ts.start, ts.stop, Ip, I.rs, Pp, P.rs, P.ps, \
                 coef, g, ntx, ntiles);                                                                 \
    }
    if (!staged) {
        GF_COEFF(8, false)  // large r': only the row sums live in LDS
    } else {
        switch (t.coeff_th) {
            case 8: GF_COEFF(8, true) break;
            case 16: GF_COEFF(16, true) break;
            case 24: GF_COEFF(24, true) break;
            default: GF_COEFF(32, true) break;
        }
    }
#undef GF_COEFF
    return hipGetLastError();
}

template <typename T>
hipError_t coeff_t(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                   hipStream_t st, const Stamp &ts, bool p_low) {
    if (g.s == 1) return coeff_tk<T, kSubId, kSubId>(I, P, coef, g, t, st, ts);
    if (g.sub == GF_SUB_NEAREST || (g.s & 1))
        return p_low ? coeff_tk<T, kSubNear, kSubId>(I, P, coef, g, t, st, ts)
                     : coeff_tk<T, kSubNear, kSubNear>(I, P, coef, g, t, st, ts);
    return p_low ? coeff_tk<T, kSubLin, kSubId>(I, P, coef, g, t, st, ts)
                 : coeff_tk<T, kSubLin, kSubLin>(I, P, coef, g, t, st, ts);
}

template <typename T, int CC, bool EPI>
hipError_t output_cc(const View &I, const View &Q, const float *mean, const Geo &g, int c0, bool vec,
                     hipStream_t st, hipEvent_t e0, hipEvent_t e1, const Detail &dt) {
    const int ntx = (g.W + kOutTileW - 1) / kOutTileW;
    const int nty = (g.H + 4 * kOutRows - 1) / (4 * kOutRows);
    const int ntiles = ntx * nty;
    const T *Ip = (const T *)I.data;
    T *Qp = (T *)Q.data + (int64_t)c0 * Q.ps;
    const T *Pp = EPI ? (const T *)dt.p.data + (int64_t)c0 * dt.p.ps : nullptr;
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_OUT(SS)                                                                                       \
    launch_k(k_output<T, CC, SS, EPI>, grid, block, 0, st, e0, e1, Ip, I.rs, Qp, Q.rs, Q.ps, mean, g, c0, ntx, \
             ntiles, (int)vec, Pp, dt.p.rs, dt.p.ps, dt.gain)
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
hipError_t output_te(const View &I, const View &Q, const float *mean, const Geo &g, bool vec,
                     hipStream_t st, const Stamp &ts, const Detail &dt) {
    for (int c0 = 0; c0 < g.C; c0 += 3) {
        const int cc = g.C - c0 < 3 ? g.C - c0 : 3;
        const hipEvent_t e0 = c0 == 0 ? ts.start : nullptr, e1 = c0 + 3 >= g.C ? ts.stop : nullptr;
        hipError_t e = cc == 3 ? output_cc<T, 3, EPI>(I, Q, mean, g, c0, vec, st, e0, e1, dt)
                     : cc == 2 ? output_cc<T, 2, EPI>(I, Q, mean, g, c0, vec, st, e0, e1, dt)
                               : output_cc<T, 1, EPI>(I, Q, mean, g, c0, vec, st, e0, e1, dt);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t output_t(const View &I, const View &Q, const float *mean, const Geo &g, bool vec,
                    hipStream_t st, const Stamp &ts, const Detail &dt) {
    return dt.p.data ? output_te<T, true>(I, Q, mean, g, vec, st, ts, dt)
                     : output_te<T, false>(I, Q, mean, g, vec, st, ts, dt);
}

}  // namespace

// Staged coefficient tiles when they fit; otherwise unstaged 8-row tiles.
bool coeff_staged(const TileCfg &t, int R) { return dev::coeff_tile_lds(t.coeff_th, R, true) <= kLdsLimit; }
size_t coeff_lds_bytes(const TileCfg &t, int R) {
    return coeff_staged(t, R) ? dev::coeff_tile_lds(t.coeff_th, R, true) : dev::coeff_tile_lds(8, R, false);
}
size_t box_lds_bytes(const TileCfg &t, int R) { return dev::box_tile_lds(t.box_th, R); }

hipError_t launch_coeff(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g,
                        const TileCfg &t, hipStream_t st, const Stamp &ts, bool p_low) {
    switch (dt) {
        case GF_F32: return coeff_t<float>(I, P, coef, g, t, st, ts, p_low);
        case GF_F16: return coeff_t<_Float16>(I, P, coef, g, t, st, ts, p_low);
        case GF_BF16: return coeff_t<dev::bf16>(I, P, coef, g, t, st, ts, p_low);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_box(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st,
                      const Stamp &ts) {
    const int ntx = (g.Wl + kTileW - 1) / kTileW, nty = (g.Hl + t.box_th - 1) / t.box_th;
    const int ntiles = ntx * nty;
    const size_t lds = box_lds_bytes(t, g.R);
    const dim3 grid(grid8(ntiles), 2 * g.C), block(kThreads);
#define GF_BOX(TH)                                                                            \
    {                                                                                         \
        allow_lds(k_box<TH>, lds);                                                            \
        launch_k(k_box<TH>, grid, block, lds, st, ts.start, ts.stop, src, dst, g, ntx, ntiles);  \
    }
    switch (t.box_th) {
        case 8: GF_BOX(8) break;
        case 16: GF_BOX(16) break;
        case 24: GF_BOX(24) break;
        default: GF_BOX(32) break;
    }
#undef GF_BOX
    return hipGetLastError();
}

hipError_t launch_output(gf_dtype dt, const View &I, const View &Q, const float *mean, const Geo &g,
                         const TileCfg &, bool vec, hipStream_t st, const Stamp &ts, const Detail &detail) {
    switch (dt) {
        case GF_F32: return output_t<float>(I, Q, mean, g, vec, st, ts, detail);
        case GF_F16: return output_t<_Float16>(I, Q, mean, g, vec, st, ts, detail);
        case GF_BF16: return output_t<dev::bf16>(I, Q, mean, g, vec, st, ts, detail);
    }
    return hipErrorInvalidValue;
}

}  // namespace gf
