// Per-image kernels of the guided filter with a colour (three-channel)
// guide, and their host launchers:
//   k_coeff_color  (grid: low-res tiles)            steps 1-4 -> a_0, a_1, a_2, b per channel
//   k_box          (grid: low-res tiles x 4C maps)  step 5 (the gray path's box tiles)
//   k_output_color (grid: full-res 1024 x 4 blocks) steps 6-7 -> q
// The tile code lives in gf_color.h.
#include "gf_color.h"
#include "gf_window_kernels.h"

namespace gf {
namespace {

template <typename T, int K, int KP, int TH, int BD>
__global__ __launch_bounds__(kThreads) void k_coeff_color(const T *__restrict__ I, int64_t Irs, int64_t Ips,
                                                          const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                                          float *__restrict__ coef, Geo g, int ntx, int ntiles) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    coeff_tile_color<T, K, TH, BD, KP>(I, Irs, Ips, P, Prs, Pps, coef, g, (tile / ntx) * TH,
                                       (tile % ntx) * kTileW, lds_d);
}

// One workgroup = 4 waves side by side = a 1024-column x 4-row block of q
// (EPI: of the detail-enhanced e, reading the matching block of p).
template <typename T, int S, bool EPI>
__global__ __launch_bounds__(kThreads) void k_output_color(const T *__restrict__ I, int64_t Irs, int64_t Ips,
                                                           T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                           const float *__restrict__ M, Geo g, int ntx, int ntiles,
                                                           const T *__restrict__ P, int64_t Prs,
                                                           int64_t Pps, float gain) {
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    output_rows_color<T, S, EPI>(I, Irs, Ips, Q, Qrs, Qps, M, g, (tile / ntx) * kColorRows,
                                 ((tile % ntx) * 4 + wave_id()) * 256, P, Prs, Pps, gain);
}

template <typename T, int K, int KP, int BD>
hipError_t coeff_color_tk(const View &I, const View &P, float *coef, const Geo &g, int th, hipStream_t st,
                          const Stamp &ts) {
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
    const int ntx = (g.Wl + kTileW - 1) / kTileW, nty = (g.Hl + th - 1) / th;
    const int ntiles = ntx * nty;
    const size_t lds = color_tile_lds(th, g.R);
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_CC(TH)                                                                                           \
    {                                                                                                        \
        allow_lds(k_coeff_color<T, K, KP, TH, BD>, lds);                                                     \
        launch_k(k_coeff_color<T, K, KP, TH, BD>, grid, block, lds, st, ts.start, ts.stop, Ip, I.rs, I.ps, Pp,  \
                 P.rs, P.ps, coef, g, ntx, ntiles);                                                          \
    }
    if (th == 16) GF_CC(16)
    else GF_CC(8)
#undef GF_CC
    return hipGetLastError();
}

template <typename T, int K, int KP>
hipError_t coeff_color_k(const View &I, const View &P, float *coef, const Geo &g, int th, hipStream_t st,
                         const Stamp &ts) {
    return g.border == GF_BORDER_CLIP ? coeff_color_tk<T, K, KP, kClip>(I, P, coef, g, th, st, ts)
                                      : coeff_color_tk<T, K, KP, kPadded>(I, P, coef, g, th, st, ts);
}

template <typename T>
hipError_t coeff_color_t(const View &I, const View &P, float *coef, const Geo &g, int th, hipStream_t st,
                         const Stamp &ts, bool p_low) {
    if (g.s == 1) return coeff_color_k<T, kSubId, kSubId>(I, P, coef, g, th, st, ts);
    if (g.sub == GF_SUB_AREA) return hipErrorInvalidValue;  // area: launch_area, then the low-res form
    if (g.sub == GF_SUB_NEAREST || (g.s & 1))
        return p_low ? coeff_color_k<T, kSubNear, kSubId>(I, P, coef, g, th, st, ts)
                     : coeff_color_k<T, kSubNear, kSubNear>(I, P, coef, g, th, st, ts);
    return p_low ? coeff_color_k<T, kSubLin, kSubId>(I, P, coef, g, th, st, ts)
                 : coeff_color_k<T, kSubLin, kSubLin>(I, P, coef, g, th, st, ts);
}

template <typename T, bool EPI>
hipError_t output_color_t(const View &I, const View &Q, const float *mean, const Geo &g, hipStream_t st,
                          const Stamp &ts, const Detail &dt) {
    const int ntx = (g.W + 1023) / 1024, nty = (g.H + kColorRows - 1) / kColorRows;
    const int ntiles = ntx * nty;
    const T *Ip = (const T *)I.data;
    T *Qp = (T *)Q.data;
    const dim3 grid(grid8(ntiles)), block(kThreads);
    const T *Pp = (const T *)dt.p.data;
#define GF_OC(SS)                                                                                             \
    launch_k(k_output_color<T, SS, EPI>, grid, block, 0, st, ts.start, ts.stop, Ip, I.rs, I.ps, Qp, Q.rs, Q.ps, mean, \
             g, ntx, ntiles, Pp, dt.p.rs, dt.p.ps, dt.gain)
    switch (g.s) {
        case 1: GF_OC(1); break;
        case 2: GF_OC(2); break;
        case 4: GF_OC(4); break;
        case 8: GF_OC(8); break;
        default: GF_OC(0); break;
    }
#undef GF_OC
    return hipGetLastError();
}

}  // namespace

hipError_t launch_coeff_color(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                              hipStream_t st, const Stamp &ts, bool p_low) {
    const int th = color_tile_h(t, g.R);
    if (!th) return hipErrorInvalidValue;
    switch (dt) {
        case GF_F32: return coeff_color_t<float>(I, P, coef, g, th, st, ts, p_low);
        case GF_F16: return coeff_color_t<_Float16>(I, P, coef, g, th, st, ts, p_low);
        case GF_BF16: return coeff_color_t<dev::bf16>(I, P, coef, g, th, st, ts, p_low);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_coeff_color_lowres(const float *Il, const float *Pl, float *coef, const Geo &g, const TileCfg &t,
                                     hipStream_t st, const Stamp &ts) {
    const int th = color_tile_h(t, g.R);
    if (!th) return hipErrorInvalidValue;
    const View vI{(void *)Il, g.lrs, g.lps}, vP{(void *)Pl, g.lrs, g.lps};
    return coeff_color_k<float, kSubId, kSubId>(vI, vP, coef, g, th, st, ts);
}

template <typename T>
hipError_t output_color_e(const View &I, const View &Q, const float *mean, const Geo &g, hipStream_t st,
                          const Stamp &ts, const Detail &dt) {
    return dt.p.data ? output_color_t<T, true>(I, Q, mean, g, st, ts, dt)
                     : output_color_t<T, false>(I, Q, mean, g, st, ts, dt);
}

hipError_t launch_output_color(gf_dtype dt, const View &I, const View &Q, const float *mean, const Geo &g,
                               hipStream_t st, const Stamp &ts, const Detail &detail) {
    switch (dt) {
        case GF_F32: return output_color_e<float>(I, Q, mean, g, st, ts, detail);
        case GF_F16: return output_color_e<_Float16>(I, Q, mean, g, st, ts, detail);
        case GF_BF16: return output_color_e<dev::bf16>(I, Q, mean, g, st, ts, detail);
    }
    return hipErrorInvalidValue;
}

}  // namespace gf
