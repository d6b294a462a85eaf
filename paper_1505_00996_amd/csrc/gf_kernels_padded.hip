// The window-sum kernels of the per-image path for the padded borders
// (replicate, reflect-101): the same tiles as the clip-normalised kernels of
// gf_kernels.hip, instantiated with the border class kPadded in a
// translation unit of their own.
#include "gf_window_kernels.h"

namespace gf {

hipError_t launch_coeff_padded(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g,
                               const TileCfg &t, hipStream_t st, const Stamp &ts, bool p_low) {
    return coeff_dt<kPadded>(dt, I, P, coef, g, t, st, ts, p_low);
}

hipError_t launch_coeff_lowres_padded(const float *Il, const float *Pl, float *coef, const Geo &g,
                                      const TileCfg &t, hipStream_t st, const Stamp &ts) {
    return coeff_lowres<kPadded>(Il, Pl, coef, g, t, st, ts);
}

hipError_t launch_box_padded(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st,
                             const Stamp &ts) {
    return box_b<kPadded>(src, dst, g, t, st, ts);
}

}  // namespace gf
