// Box means of a, b fused into the output pass (Algorithm 2 steps 5-7) for
// ratios s in {2, 4, 8} and a gray guide.
//
// A workgroup covers a 32-row x (64 PX)-column block of q, its four waves
// stacked (8 rows each, PX pixels per lane as in output_rows).  Channel by
// channel it reads the low-res a_c, b_c under the block with an r' halo,
// forms in LDS the box means mean_a, mean_b of the low-res patch the block
// interpolates from, and runs the arithmetic of output_rows on them.  The
// separate box-mean pass (writing mean_a, mean_b) and its re-read are gone:
// the HBM traffic of those maps drops from four passes to one.
//
// The means are formed with box_tile's operations in box_tile's order: row
// sums over runs of kRun outputs that start at multiples of kRun (the
// (2r'+1)-term sum, then add-in/take-out steps), and column sums over runs of
// LC = box_th / 4 rows that start at multiples of LC, then one multiply by
// the reciprocal of the window's pixel count.  Which runs a value belongs to
// depends only on its position, so every mean equals, bit for bit, what
// box_tile writes with tiles of box_th rows, whatever block computes it; so
// q equals that of the three-pass path with the same tiles.  The block
// computes the whole runs that cover its patch.
#pragma once

#include "gf_device.h"

namespace gf {

namespace dev {

// Four consecutive values of row `row` (map row index y, already resolved
// for padded borders) of a low-res plane at map columns x .. x+3, as the
// region fill of box_tile stages them: outside the map 0 (kClip: the value
// at a clamped position times 0) or the padded border's value (kPadded).
// fy: 1 for a row inside the map, 0 outside (kClip only).
template <int BD, bool COH>
__device__ __forceinline__ f32x4 ob_load4(const float *__restrict__ row, int x, float fy, const Geo &g) {
    f32x4 v;
    if (!COH && x >= 0 && x + 3 < g.Wl) {
        v = *(const f32x4e *)(row + x);
        if constexpr (BD == kClip) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = v[e] * fy;
        }
        return v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int xe = x + e;
        if constexpr (BD == kClip) {
            const bool in = xe >= 0 && xe < g.Wl;
            v[e] = ldp<COH>(row + clampi(xe, 0, g.Wl - 1)) * (in ? fy : 0.f);
        } else {
            v[e] = ldp<COH>(row + pad_index(xe, g.Wl, g.border, g.refl_w));
        }
    }
    return v;
}

// Row sums (box_tile's row pass) of one region row of plane S over the
// kRun computed columns starting at map column xr (a multiple of kRun):
// out[t] = sum of the map values at xr + t - R .. xr + t + R.
template <int BD, bool COH>
__device__ __forceinline__ void ob_row_run(const float *__restrict__ S, int y, int xr, const Geo &g,
                                           float (&out)[kRun]) {
    const int R = g.R;
    float fy = 1.f;
    int yy;
    if constexpr (BD == kClip) {
        fy = (y >= 0 && y < g.Hl) ? 1.f : 0.f;
        yy = clampi(y, 0, g.Hl - 1);
    } else {
        yy = pad_index(y, g.Hl, g.border, g.refl_h);
    }
    const float *row = S + (int64_t)yy * g.lrs;
    const int xs = xr - R;  // map column of window value 0
    // window values 0..7 (also the values taken out by the run's steps)
    const f32x4 w0 = ob_load4<BD, COH>(row, xs, fy, g), w1 = ob_load4<BD, COH>(row, xs + 4, fy, g);
    // values 2R+1 .. 2R+8 (added by the steps)
    const f32x4 n0 = ob_load4<BD, COH>(row, xs + 2 * R + 1, fy, g);
    const f32x4 n1 = ob_load4<BD, COH>(row, xs + 2 * R + 5, fy, g);
    const float vout[8] = {w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
    const float vin[8] = {n0[0], n0[1], n0[2], n0[3], n1[0], n1[1], n1[2], n1[3]};
    float A = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k <= 2 * R) A += vout[k];
    for (int q = 8; q <= 2 * R; q += 4) {
        const f32x4 w = ob_load4<BD, COH>(row, xs + q, fy, g);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (q + e <= 2 * R) A += w[e];
    }
    out[0] = A;
#pragma unroll
    for (int t = 1; t < kRun; ++t) {
        A += vin[t - 1] - vout[t - 1];
        out[t] = A;
    }
}

// One fused block: channels [cb, ce) of q (planes Q + c*Qps) for the block
// at (y0, xw); a_c at coef + c*lps, b_c at coef + (C+c)*lps.  LC = box_th/4.
// Called by the whole workgroup (barriers inside); lds holds outbox_lds(...)
// bytes.  EPI: detail enhancement as in output_rows.
template <typename T, int S, bool EPI, int PX, int BD, bool COH>
__device__ __forceinline__ void outbox_block(const T *__restrict__ I, int64_t Irs, T *__restrict__ Q, int64_t Qrs,
                                             int64_t Qps, const float *__restrict__ coef, const Geo &g, int cb,
                                             int ce, int y0, int xw, int LC, float *lds,
                                             const T *__restrict__ P = nullptr, int64_t Prs = 0, int64_t Pps = 0,
                                             float gain = 0.f) {
    static_assert(S == 2 || S == 4 || S == 8, "fused blocks take s in {2, 4, 8}");
    static_assert(PX == 4 || PX == 8, "4 or 8 pixels per lane");
    constexpr int ROWS = kOutRows;
    const int R = g.R;
    const int lane = threadIdx.x & 63;
    const int yb = y0 + wave_id() * ROWS, x0 = xw + lane * PX;
    const int nrows = max(0, min(ROWS, g.H - yb));
    const bool act = x0 < g.W && nrows > 0;
    const bool full = x0 + PX - 1 < g.W;

    // the patch the block interpolates from, and the whole runs computed
    const int yl = min(y0 + kObRows - 1, g.H - 1), xl = min(xw + 64 * PX - 1, g.W - 1);
    const int py0 = clampi(floordiv(2 * y0 + 1 - S, 2 * S), 0, g.Hl - 1);
    const int py1 = clampi(floordiv(2 * yl + 1 - S, 2 * S) + 1, 0, g.Hl - 1);
    const int px0 = clampi(floordiv(2 * xw + 1 - S, 2 * S), 0, g.Wl - 1);
    const int px1 = clampi(floordiv(2 * xl + 1 - S, 2 * S) + 1, 0, g.Wl - 1);
    const int gy = (py0 / LC) * LC, nrc = (py1 / LC + 1) * LC - gy;
    const int gx = (px0 / kRun) * kRun, ncc = (px1 / kRun + 1) * kRun - gx;
    const int rh = nrc + 2 * R, hsw = ncc + 1;
    float *Ha = lds, *Hb = Ha + rh * hsw, *Pa = Hb + rh * hsw, *Pb = Pa + nrc * hsw;

    typedef PixRow<T, PX> Row;
    auto load_row = [&](const T *plane, int64_t rs, int y, Row &r) {
        ld_row<T, PX>(r, plane + (int64_t)y * rs + x0, full, g.W - x0);
    };
    Row iv[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        if (act && i < nrows) load_row(I, Irs, yb + i, iv[i]);
        else iv[i].zero();
    }
    auto store_q = [&](T *plane, int y, const float *v) {
        T *row = plane + (int64_t)y * Qrs + x0;
        if (full) {
            stv<PX>(row, v);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j)
                if (x0 + j < g.W) st1(row + j, v[j]);
        }
    };
    Row pv[EPI ? ROWS : 1];
    pv[0].zero();

    // taps and weights of output_rows (compile-time ratio), as offsets into
    // the patches
    constexpr int NL = cfloor_u(ROWS - 1, S) - cfloor_u(0, S) + 2;
    constexpr int NC = cfloor_u(PX - 1, S) - cfloor_u(0, S) + 2;
    const int base_y = floordiv(2 * yb + 1 - S, 2 * S);
    const int base_x = floordiv(2 * x0 + 1 - S, 2 * S);
    int roff[NL], coff[NC];
#pragma unroll
    for (int m = 0; m < NL; ++m) roff[m] = (clampi(base_y + m, 0, g.Hl - 1) - gy) * hsw;
#pragma unroll
    for (int m = 0; m < NC; ++m) coff[m] = clampi(base_x + m, 0, g.Wl - 1) - gx;
    constexpr bool XPHASE = S == 8 && PX == 4;
    float wx[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j)
        wx[j] = XPHASE ? (float)((2 * ((x0 & 7) + j) + 1 - 8) & 15) * (1.0f / 16.0f) : cfrac_u(j, S);

    const int nruns_x = ncc / kRun;
#pragma unroll 1
    for (int c = cb; c < ce; ++c) {
        const float *Sa = coef + (int64_t)c * g.lps, *Sb = coef + (int64_t)(g.C + c) * g.lps;
        // row sums of every region row over the computed columns (lanes take
        // consecutive rows of one run: the row-sum writes stride hsw, odd)
        for (int it = threadIdx.x; it < rh * nruns_x; it += kThreads) {
            const int m = it / rh, ry = it - m * rh;
            const int y = gy - R + ry, xr = gx + m * kRun;
            float ra[kRun], rb[kRun];
            ob_row_run<BD, COH>(Sa, y, xr, g, ra);
            ob_row_run<BD, COH>(Sb, y, xr, g, rb);
            float *ha = Ha + ry * hsw + m * kRun, *hb = Hb + ry * hsw + m * kRun;
#pragma unroll
            for (int t = 0; t < kRun; ++t) {
                ha[t] = ra[t];
                hb[t] = rb[t];
            }
        }
        lds_sync();  // row sums done; every lane has finished reading the previous patches
        // column sums over runs of LC rows, divided by the window's count
        for (int it = threadIdx.x; it < ncc * (nrc / LC); it += kThreads) {
            const int m = it / ncc, j = it - m * ncc;
            const int i0 = m * LC, lx = gx + j;
            const int nx = window_len<BD>(lx, R, g.Wl);
            float A = 0.f, B = 0.f;
            for (int k = 0; k <= 2 * R; ++k) {
                A += Ha[(i0 + k) * hsw + j];
                B += Hb[(i0 + k) * hsw + j];
            }
            for (int t = 0; t < LC; ++t) {
                if (t) {
                    A += Ha[(i0 + t + 2 * R) * hsw + j] - Ha[(i0 + t - 1) * hsw + j];
                    B += Hb[(i0 + t + 2 * R) * hsw + j] - Hb[(i0 + t - 1) * hsw + j];
                }
                const int ly = gy + i0 + t;
                float ma = 0.f, mb = 0.f;  // positions past the map are never read
                if (ly < g.Hl && lx < g.Wl) {
                    const float rn = rcp((float)(window_len<BD>(ly, R, g.Hl) * nx));
                    ma = A * rn;
                    mb = B * rn;
                }
                Pa[(i0 + t) * hsw + j] = ma;
                Pb[(i0 + t) * hsw + j] = mb;
            }
        }
        lds_sync();  // patches of mean_a, mean_b complete
        if (act) {
            T *Qc = Q + (int64_t)c * Qps;
            if constexpr (EPI) {
                const T *Pc = P + (int64_t)c * Pps;
#pragma unroll
                for (int i = 0; i < ROWS; ++i) {
                    if (i < nrows) load_row(Pc, Prs, yb + i, pv[i]);
                    else pv[i].zero();
                }
            }
            float va[NL][NC], vb[NL][NC];
#pragma unroll
            for (int m = 0; m < NL; ++m) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    va[m][k] = Pa[roff[m] + coff[k]];
                    vb[m][k] = Pb[roff[m] + coff[k]];
                }
            }
            auto hlerp = [&](const float (&v)[NL][NC], int m, int j) -> float {
                const int k0 = XPHASE ? 0 : cfloor_u(j, S) - cfloor_u(0, S);
                return lerp(v[m][k0], v[m][k0 + 1], wx[j]);
            };
            constexpr bool HOIST = PX == 4;
            float ha[HOIST ? NL : 1][PX], hb[HOIST ? NL : 1][PX];
            if constexpr (HOIST) {
#pragma unroll
                for (int m = 0; m < NL; ++m) {
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        ha[m][j] = hlerp(va, m, j);
                        hb[m][j] = hlerp(vb, m, j);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int m0 = cfloor_u(i, S) - cfloor_u(0, S);
                    const float wy = cfrac_u(i, S);
                    float out[PX];
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        const float a0 = HOIST ? ha[m0][j] : hlerp(va, m0, j);
                        const float a1 = HOIST ? ha[m0 + 1][j] : hlerp(va, m0 + 1, j);
                        const float b0 = HOIST ? hb[m0][j] : hlerp(vb, m0, j);
                        const float b1 = HOIST ? hb[m0 + 1][j] : hlerp(vb, m0 + 1, j);
                        out[j] = madd(lerp(a0, a1, wy), iv[i].at(j), lerp(b0, b1, wy));
                    }
                    if constexpr (EPI) {
#pragma unroll
                        for (int j = 0; j < PX; ++j) out[j] = lerp(out[j], pv[i].at(j), gain);
                    }
                    store_q(Qc, yb + i, out);
                }
            }
        }
    }
}

}  // namespace dev
}  // namespace gf
