// The per-image window-sum kernels (coefficients: Algorithm 2 steps 1-4; box
// means: step 5), their launch helpers and their host launchers, templated on
// the border class (kClip, kPadded).  Included by gf_kernels.hip, which
// instantiates the clip-normalised kernels, and by gf_kernels_padded.hip,
// which instantiates the padded-border ones, so the two sets compile in
// parallel.  Everything here has internal linkage in each includer.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "gf_device.h"
#include "gf_internal.h"

namespace gf {
namespace {

using namespace dev;

template <typename T, int K, int KP, int TH, bool STAGE, int BD>
__global__ __launch_bounds__(kThreads) void k_coeff(const T *__restrict__ I, int64_t Irs,
                                                    const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                                    float *__restrict__ coef, Geo g, int ntx, int ntiles, int cpg) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    // blockIdx.y: a group of cpg channels of p
    const int cb = (int)blockIdx.y * cpg;
    coeff_tile<T, K, TH, STAGE, false, KP, BD>(I, Irs, P, Prs, Pps, coef, g, (tile / ntx) * TH,
                                               (tile % ntx) * kTileW, lds_d, cb, min(g.C, cb + cpg));
}

template <int TH, int BD>
__global__ __launch_bounds__(kThreads) void k_box(const float *__restrict__ src, float *__restrict__ dst,
                                                  Geo g, int ntx, int ntiles) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    box_tile<TH, false, BD>(src + (int64_t)blockIdx.y * g.lps, dst + (int64_t)blockIdx.y * g.lps, g,
                            (tile / ntx) * TH, (tile % ntx) * kTileW, lds_d);
}

inline int grid8(int n) { return ((n + 7) / 8) * 8; }

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

template <typename T, int K, int KP, int BD>
hipError_t coeff_tk(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                    hipStream_t st, const Stamp &ts) {
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
    const bool staged = coeff_staged(t, g.R);
    const int th = staged ? t.coeff_th : 8;  // the unstaged kernel works on 8-row tiles
    const int ntx = (g.Wl + kTileW - 1) / kTileW, nty = (g.Hl + th - 1) / th;
    const int ntiles = ntx * nty;
    const size_t lds = coeff_lds_bytes(t, g.R);
    // With fewer tiles than CUs, one workgroup per tile and channel (each
    // forms the guide's sums itself; the same bits): the 6000x4000 RGB map at
    // s = 8 (252 tiles) took 14.8 us against 17.3; with more tiles the extra
    // guide passes cost more than the shorter chains save (4000x3000 at
    // s = 4, 512 tiles: 25.1 us against 21.6).
    const int cpg = ntiles < kCUs ? 1 : g.C;
    const dim3 grid(grid8(ntiles), (g.C + cpg - 1) / cpg), block(kThreads);
#define GF_COEFF(TH, STG)                                                                                  \
    {                                                                                                       \
        allow_lds(k_coeff<T, K, KP, TH, STG, BD>, lds);                                                     \
        launch_k(k_coeff<T, K, KP, TH, STG, BD>, grid, block, lds, st, ts.start, ts.stop, Ip, I.rs, Pp, P.rs, \
                 P.ps, coef, g, ntx, ntiles, cpg);                                                          \
    }
    if (!staged) {
        GF_COEFF(8, false)  // large r': only the row sums live in LDS
    } else {
        switch (t.coeff_th) {
            case 8: GF_COEFF(8, true) break;
            case 16: GF_COEFF(16, true) break;
            case 24: GF_COEFF(24, true) break;
            case 32: GF_COEFF(32, true) break;
            case 48: GF_COEFF(48, true) break;
            default: GF_COEFF(64, true) break;
        }
    }
#undef GF_COEFF
    return hipGetLastError();
}

template <typename T, int BD>
hipError_t coeff_t(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                   hipStream_t st, const Stamp &ts, bool p_low) {
    if (g.s == 1) return coeff_tk<T, kSubId, kSubId, BD>(I, P, coef, g, t, st, ts);
    if (g.sub == GF_SUB_AREA) return hipErrorInvalidValue;  // area: launch_area, then launch_coeff_lowres
    if (g.sub == GF_SUB_NEAREST || (g.s & 1))
        return p_low ? coeff_tk<T, kSubNear, kSubId, BD>(I, P, coef, g, t, st, ts)
                     : coeff_tk<T, kSubNear, kSubNear, BD>(I, P, coef, g, t, st, ts);
    return p_low ? coeff_tk<T, kSubLin, kSubId, BD>(I, P, coef, g, t, st, ts)
                 : coeff_tk<T, kSubLin, kSubLin, BD>(I, P, coef, g, t, st, ts);
}

template <int BD>
hipError_t coeff_dt(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                    hipStream_t st, const Stamp &ts, bool p_low) {
    switch (dt) {
        case GF_F32: return coeff_t<float, BD>(I, P, coef, g, t, st, ts, p_low);
        case GF_F16: return coeff_t<_Float16, BD>(I, P, coef, g, t, st, ts, p_low);
        case GF_BF16: return coeff_t<dev::bf16, BD>(I, P, coef, g, t, st, ts, p_low);
    }
    return hipErrorInvalidValue;
}

template <int BD>
hipError_t coeff_lowres(const float *Il, const float *Pl, float *coef, const Geo &g, const TileCfg &t,
                        hipStream_t st, const Stamp &ts) {
    const View vI{(void *)Il, g.lrs, g.lps}, vP{(void *)Pl, g.lrs, g.lps};
    return coeff_tk<float, kSubId, kSubId, BD>(vI, vP, coef, g, t, st, ts);
}

template <int BD>
hipError_t box_b(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st,
                 const Stamp &ts) {
    const int ntx = (g.Wl + kTileW - 1) / kTileW, nty = (g.Hl + t.box_th - 1) / t.box_th;
    const int ntiles = ntx * nty;
    const size_t lds = box_lds_bytes(t, g.R);
    const dim3 grid(grid8(ntiles), 2 * g.C), block(kThreads);
#define GF_BOX(TH)                                                                                    \
    {                                                                                                 \
        allow_lds(k_box<TH, BD>, lds);                                                                \
        launch_k(k_box<TH, BD>, grid, block, lds, st, ts.start, ts.stop, src, dst, g, ntx, ntiles);  \
    }
    switch (t.box_th) {
        case 8: GF_BOX(8) break;
        case 16: GF_BOX(16) break;
        case 24: GF_BOX(24) break;
        case 32: GF_BOX(32) break;
        case 48: GF_BOX(48) break;
        default: GF_BOX(64) break;
    }
#undef GF_BOX
    return hipGetLastError();
}

}  // namespace
}  // namespace gf
