// Per-image kernel of Algorithm 2 steps 5-7 fused (gf_outbox.h): with it a
// fast filter at s in {2, 4, 8} with a gray guide runs as two launches,
//   k_coeff  (grid: low-res tiles)               steps 1-4 -> a, b
//   k_outbox (grid: full-res 32 x (64 PX) blocks) steps 5-7 -> q
// instead of k_coeff, k_box, k_output.
#include "gf_outbox.h"
#include "gf_window_kernels.h"

namespace gf {
namespace {

using namespace dev;

// One workgroup = one 32-row x (64 PX)-column block of q, all C channels
// (EPI: of the detail-enhanced e, reading the matching block of p).
template <typename T, int S, bool EPI, int PX, int BD>
__global__ __launch_bounds__(kThreads) void k_outbox(const T *__restrict__ I, int64_t Irs, T *__restrict__ Q,
                                                     int64_t Qrs, int64_t Qps, const float *__restrict__ coef,
                                                     Geo g, int LC, int ntx, int ntiles,
                                                     const T *__restrict__ P, int64_t Prs, int64_t Pps, float gain) {
    extern __shared__ double lds_d[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    outbox_block<T, S, EPI, PX, BD, false>(I, Irs, Q, Qrs, Qps, coef, g, 0, g.C, (tile / ntx) * kObRows,
                                           (tile % ntx) * (64 * PX), LC, (float *)lds_d, P, Prs, Pps, gain);
}

template <typename T, int S, bool EPI, int PX, int BD>
hipError_t outbox_go(const View &I, const View &Q, const float *coef, const Geo &g, int LC, hipStream_t st,
                     const Stamp &ts, const Detail &dt) {
    const int tw = 64 * PX;
    const int ntx = (g.W + tw - 1) / tw, nty = (g.H + kObRows - 1) / kObRows;
    const int ntiles = ntx * nty;
    const size_t lds = outbox_lds(S, g.R, LC, PX);
    allow_lds(k_outbox<T, S, EPI, PX, BD>, lds);
    launch_k(k_outbox<T, S, EPI, PX, BD>, dim3(grid8(ntiles)), dim3(kThreads), lds, st, ts.start, ts.stop,
             (const T *)I.data, I.rs, (T *)Q.data, Q.rs, Q.ps, coef, g, LC, ntx, ntiles,
             EPI ? (const T *)dt.p.data : (const T *)nullptr, dt.p.rs, dt.p.ps, dt.gain);
    return hipGetLastError();
}

template <typename T, int S, bool EPI, int BD>
hipError_t outbox_px(int px, const View &I, const View &Q, const float *coef, const Geo &g, int LC, hipStream_t st,
                     const Stamp &ts, const Detail &dt) {
    if constexpr (sizeof(T) == 2) {
        if (px == 8) return outbox_go<T, S, EPI, 8, BD>(I, Q, coef, g, LC, st, ts, dt);
    }
    if (px != 4) return hipErrorInvalidValue;
    return outbox_go<T, S, EPI, 4, BD>(I, Q, coef, g, LC, st, ts, dt);
}

template <typename T, bool EPI, int BD>
hipError_t outbox_s(int px, const View &I, const View &Q, const float *coef, const Geo &g, int LC, hipStream_t st,
                    const Stamp &ts, const Detail &dt) {
    switch (g.s) {
        case 2: return outbox_px<T, 2, EPI, BD>(px, I, Q, coef, g, LC, st, ts, dt);
        case 4: return outbox_px<T, 4, EPI, BD>(px, I, Q, coef, g, LC, st, ts, dt);
        case 8: return outbox_px<T, 8, EPI, BD>(px, I, Q, coef, g, LC, st, ts, dt);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t outbox_t(int px, const View &I, const View &Q, const float *coef, const Geo &g, int LC, hipStream_t st,
                    const Stamp &ts, const Detail &dt) {
    const bool epi = dt.p.data != nullptr, pad = g.border != GF_BORDER_CLIP;
    if (epi) return pad ? outbox_s<T, true, kPadded>(px, I, Q, coef, g, LC, st, ts, dt)
                        : outbox_s<T, true, kClip>(px, I, Q, coef, g, LC, st, ts, dt);
    return pad ? outbox_s<T, false, kPadded>(px, I, Q, coef, g, LC, st, ts, dt)
               : outbox_s<T, false, kClip>(px, I, Q, coef, g, LC, st, ts, dt);
}

}  // namespace

hipError_t launch_outbox(gf_dtype dt, const View &I, const View &Q, const float *coef, const Geo &g,
                         const TileCfg &t, int px, hipStream_t st, const Stamp &ts, const Detail &detail) {
    const int LC = t.box_th / 4;
    switch (dt) {
        case GF_F32: return outbox_t<float>(px, I, Q, coef, g, LC, st, ts, detail);
        case GF_F16: return outbox_t<_Float16>(px, I, Q, coef, g, LC, st, ts, detail);
        case GF_BF16: return outbox_t<dev::bf16>(px, I, Q, coef, g, LC, st, ts, detail);
    }
    return hipErrorInvalidValue;
}

}  // namespace gf
