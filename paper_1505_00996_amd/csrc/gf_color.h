// Device code of the guided filter with a colour (three-channel) guide: the
// tile functions of the coefficient pass and of the output pass.  The model
// per window is q = a.I + b with a a 3-vector; a = (Sigma + eps U)^-1 cov(I, p)
// and b = mean(p) - a.mean(I), Sigma the 3x3 covariance of I in the window.
// The box means of a and b are the gray path's box tiles over 4C planes.
//
// Map layout (workspace, low resolution): a_j of channel c at plane 3c + j
// (j = 0, 1, 2), b of channel c at plane 3C + c; the box means in the same
// order after them.
#pragma once

#include "gf_device.h"

namespace gf {
namespace dev {

// x = M^-1 y for the symmetric 3x3 M = [[m00 m01 m02] [m01 m11 m12] [m02 m12 m22]],
// by its adjugate and determinant (FP64).
__device__ __forceinline__ void solve3_sym(double m00, double m01, double m02, double m11, double m12,
                                           double m22, const double y[3], double x[3]) {
    const double c00 = m11 * m22 - m12 * m12;
    const double c01 = m02 * m12 - m01 * m22;
    const double c02 = m01 * m12 - m02 * m11;
    const double c11 = m00 * m22 - m02 * m02;
    const double c12 = m01 * m02 - m00 * m12;
    const double c22 = m00 * m11 - m01 * m01;
    const double rd = 1.0 / (m00 * c00 + m01 * c01 + m02 * c02);
    x[0] = (c00 * y[0] + c01 * y[1] + c02 * y[2]) * rd;
    x[1] = (c01 * y[0] + c11 * y[1] + c12 * y[2]) * rd;
    x[2] = (c02 * y[0] + c12 * y[1] + c22 * y[2]) * rd;
}

// One TH x 64 tile of a_0, a_1, a_2 and b (low-res) for every channel of p,
// colour guide I (planes I + j*Ips), sampling kind K, border class BD.  The
// staged regions hold u_j = I'_j - c_j (shifted by the tile's first sample)
// and v = p' - c_p.  Window sums are FP64 (products of FP32 samples are
// exact in FP64): each pass is a row pass writing two row-sum planes, then a
// column pass summing them into registers.  Five passes give the guide's
// nine sums (S_j, S_jk) once for all channels; two more per channel give
// S_v and S_jv (channel 0's S_1v rides in the fifth).  Then per pixel, with
// n the window's sample count, n^2 Sigma_jk = n S_jk - S_j S_k and
// n^2 cov_j = n S_jv - S_j S_v, and a = (n^2 Sigma + n^2 eps U)^-1 (n^2 cov),
// solved in FP64.
// KP: how p is sampled -- like I, or kSubId when p is given at low
// resolution (joint upsampling).
template <typename T, int K, int TH, int BD, int KP = K>
__device__ __forceinline__ void coeff_tile_color(const T *__restrict__ I, int64_t Irs, int64_t Ips,
                                                 const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                                 float *__restrict__ coef, const Geo &g, int ty0, int tx0,
                                                 void *lds) {
    constexpr int LC = TH / 4;  // output rows per thread in the column pass
    const int R = g.R, SH = TH + 2 * R, SW = kTileW + 2 * R, SWp = region_stride(R);
    const int plane = SH * kRowW, region = SH * SWp;
    double *rA = (double *)lds, *rB = rA + plane;
    float *sU0 = (float *)(rB + plane), *sU1 = sU0 + region, *sU2 = sU1 + region, *sV = sU2 + region;
    const int oy = ty0 - R, ox = tx0 - R;
    const int lane = threadIdx.x & 63, wave = wave_id();

    // the shifted sample of an image at region position (ry, rx); outside
    // the map 0 (kClip, a product rather than a select: see coeff_tile) or
    // the border extension's sample (kPadded)
    auto gsample = [&](auto kind, const T *img, int64_t rs, float c, int ry, int rx) -> float {
        constexpr int KK = decltype(kind)::value;
        const int ly = oy + ry, lx = ox + rx;
        if constexpr (BD == kClip) {
            const bool in = ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
            const float v = sample_rc<KK>(img, rs, taps<KK>(clampi(ly, 0, g.Hl - 1), g.s, g.H),
                                          taps<KK>(clampi(lx, 0, g.Wl - 1), g.s, g.W));
            return (v - c) * (in ? 1.f : 0.f);
        } else {
            const float v = sample_rc<KK>(img, rs, taps<KK>(pad_index(ly, g.Hl, g.border, g.refl_h), g.s, g.H),
                                          taps<KK>(pad_index(lx, g.Wl, g.border, g.refl_w), g.s, g.W));
            return v - c;
        }
    };
    using KI = std::integral_constant<int, K>;
    using KQ = std::integral_constant<int, KP>;
    const T *I0 = I, *I1 = I + Ips, *I2 = I + 2 * Ips;
    const float c0 = sample<K>(I0, Irs, ty0, tx0, g), c1 = sample<K>(I1, Irs, ty0, tx0, g),
                c2 = sample<K>(I2, Irs, ty0, tx0, g);
    fill_tile2(sU0, sU1, SH, SW, SWp, [&](int ry, int rx) { return gsample(KI{}, I0, Irs, c0, ry, rx); },
               [&](int ry, int rx) { return gsample(KI{}, I1, Irs, c1, ry, rx); });
    float cP = sample<KP>(P, Prs, ty0, tx0, g);
    fill_tile2(sU2, sV, SH, SW, SWp, [&](int ry, int rx) { return gsample(KI{}, I2, Irs, c2, ry, rx); },
               [&](int ry, int rx) { return gsample(KQ{}, P, Prs, cP, ry, rx); });
    lds_sync();

    // Row pass: rA = sum X*Y and rB = sum X*Z over each window of a run of
    // kRun outputs (HY / HZ false: the factor 1 instead of Y / Z).  Lanes
    // take consecutive rows of a run (bank-conflict-free, as in coeff_tile);
    // every read of a run comes before its writes.
    auto row_pass = [&](auto hy, auto hz, const float *X, const float *Y, const float *Z) {
        constexpr bool HY = decltype(hy)::value, HZ = decltype(hz)::value;
        for (int it = threadIdx.x; it < SH * (kTileW / kRun); it += kThreads) {
            const int j0 = (it / SH) * kRun, ry = it - (it / SH) * SH;
            const int o = ry * SWp + j0;
            auto xy = [&](int k) -> double { return HY ? (double)X[o + k] * (double)Y[o + k] : (double)X[o + k]; };
            auto xz = [&](int k) -> double { return HZ ? (double)X[o + k] * (double)Z[o + k] : (double)X[o + k]; };
            double ain[kRun], aout[kRun], bin[kRun], bout[kRun];
#pragma unroll
            for (int t = 1; t < kRun; ++t) {
                ain[t] = xy(t + 2 * R);
                aout[t] = xy(t - 1);
                bin[t] = xz(t + 2 * R);
                bout[t] = xz(t - 1);
            }
            double A = 0.0, B = 0.0;
#pragma unroll 8
            for (int k = 0; k <= 2 * R; ++k) {
                A += xy(k);
                B += xz(k);
            }
            double ra[kRun], rb[kRun];
            ra[0] = A;
            rb[0] = B;
#pragma unroll
            for (int t = 1; t < kRun; ++t) {
                A += ain[t] - aout[t];
                B += bin[t] - bout[t];
                ra[t] = A;
                rb[t] = B;
            }
            double *oa = rA + ry * kRowW + j0, *ob = rB + ry * kRowW + j0;
#pragma unroll
            for (int t = 0; t < kRun; ++t) {
                oa[t] = ra[t];
                ob[t] = rb[t];
            }
        }
    };
    const int col = lane, r0 = wave * LC;
    // Column pass: the window sums of rA and rB for this thread's LC rows.
    auto col_pass = [&](double *SA, double *SB) {
        double A = 0.0, B = 0.0;
#pragma unroll 8
        for (int k = 0; k <= 2 * R; ++k) {
            A += rA[(r0 + k) * kRowW + col];
            B += rB[(r0 + k) * kRowW + col];
        }
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            if (t) {
                A += rA[(r0 + t + 2 * R) * kRowW + col] - rA[(r0 + t - 1) * kRowW + col];
                B += rB[(r0 + t + 2 * R) * kRowW + col] - rB[(r0 + t - 1) * kRowW + col];
            }
            SA[t] = A;
            SB[t] = B;
        }
    };
    auto pass = [&](auto hy, const float *X, const float *Y, const float *Z, double *SA, double *SB) {
        row_pass(hy, std::true_type{}, X, Y, Z);
        lds_sync();
        col_pass(SA, SB);
        lds_sync();  // rA, rB free for the next row pass
    };

    // the guide's nine sums (the fifth pass also takes channel 0's sum of u1 v)
    double S0[LC], S1[LC], S2[LC], S00[LC], S11[LC], S22[LC], S01[LC], S02[LC], S12[LC];
    double Sv[LC], S0v[LC], S1v[LC], S2v[LC], unused[LC];
    using one = std::false_type;
    using prod = std::true_type;
    pass(one{}, sU0, nullptr, sU0, S0, S00);
    pass(one{}, sU1, nullptr, sU1, S1, S11);
    pass(one{}, sU2, nullptr, sU2, S2, S22);
    pass(prod{}, sU0, sU1, sU2, S01, S02);
    pass(prod{}, sU1, sU2, sV, S12, S1v);

    const int lx = tx0 + col;
    const int nx = window_len<BD>(lx, R, g.Wl);
    const double eps = (double)g.eps;
    for (int c = 0; c < g.C; ++c) {
        if (c) {
            // sV is free: the last row pass that read it ended at a barrier
            const T *Pc = P + (int64_t)c * Pps;
            cP = sample<KP>(Pc, Prs, ty0, tx0, g);
            fill_tile(sV, SH, SW, SWp, [&](int ry, int rx) { return gsample(KQ{}, Pc, Prs, cP, ry, rx); });
            lds_sync();
            pass(one{}, sV, nullptr, sU0, Sv, S0v);
            pass(prod{}, sV, sU1, sU2, S1v, S2v);
        } else {
            pass(one{}, sV, nullptr, sU0, Sv, S0v);
            pass(prod{}, sV, sU2, sU2, S2v, unused);
        }
        float *a0 = coef + (int64_t)(3 * c) * g.lps, *a1 = a0 + g.lps, *a2 = a1 + g.lps;
        float *bc = coef + (int64_t)(3 * g.C + c) * g.lps;
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            const int ly = ty0 + r0 + t;
            if (ly < g.Hl && lx < g.Wl) {
                const double n = (double)(window_len<BD>(ly, R, g.Hl) * nx);
                const double n2e = n * n * eps;
                const double m00 = fmax(n * S00[t] - S0[t] * S0[t], 0.0) + n2e;
                const double m11 = fmax(n * S11[t] - S1[t] * S1[t], 0.0) + n2e;
                const double m22 = fmax(n * S22[t] - S2[t] * S2[t], 0.0) + n2e;
                const double m01 = n * S01[t] - S0[t] * S1[t];
                const double m02 = n * S02[t] - S0[t] * S2[t];
                const double m12 = n * S12[t] - S1[t] * S2[t];
                const double y[3] = {n * S0v[t] - S0[t] * Sv[t], n * S1v[t] - S1[t] * Sv[t],
                                     n * S2v[t] - S2[t] * Sv[t]};
                double a[3];
                solve3_sym(m00, m01, m02, m11, m12, m22, y, a);
                const double rn = 1.0 / n;
                const double mp = (double)cP + Sv[t] * rn;
                const double b = mp - (a[0] * ((double)c0 + S0[t] * rn) + a[1] * ((double)c1 + S1[t] * rn) +
                                       a[2] * ((double)c2 + S2[t] * rn));
                const int64_t at = (int64_t)ly * g.lrs + lx;
                a0[at] = (float)a[0];
                a1[at] = (float)a[1];
                a2[at] = (float)a[2];
                bc[at] = (float)b;
            }
        }
    }
}

// q for every channel of p at the wave's 4 x 256 block at (yb, xw), colour
// guide I (planes I + j*Ips), four pixels per lane.  q_c = mean_a_0 I_0 +
// mean_a_1 I_1 + mean_a_2 I_2 + mean_b with the means bilinearly upsampled
// from the low-res maps M (layout above).  S: compile-time ratio (0: g.s at
// run time).  The lane first loads its 3 x 4 x 4 guide values; then per
// channel the low-res values its pixels interpolate from, and per row the
// bilinear weights and the stores.  EPI (detail enhancement): with P the
// input p (layout of Q), each output is e = q + gain (p - q), formed from the
// FP32 q before the store's rounding.
constexpr int kColorRows = 4;
template <typename T, int S, bool EPI = false>
__device__ __forceinline__ void output_rows_color(const T *__restrict__ I, int64_t Irs, int64_t Ips,
                                                  T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                  const float *__restrict__ M, const Geo &g, int yb, int xw,
                                                  const T *__restrict__ P = nullptr, int64_t Prs = 0,
                                                  int64_t Pps = 0, float gain = 0.f) {
    constexpr int ROWS = kColorRows, PX = 4;
    const int lane = threadIdx.x & 63;
    const int x0 = xw + lane * PX;
    const int nrows = min(ROWS, g.H - yb);
    if (x0 >= g.W || nrows <= 0) return;  // no barriers below
    const bool full = x0 + PX - 1 < g.W;  // one wide access per row, else element-wise
    typedef PixRow<T, PX> Row;
    Row iv[3][ROWS];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            if (i < nrows) {
                const T *base = I + (int64_t)j * Ips + (int64_t)(yb + i) * Irs;
                ld_row<T, PX>(iv[j][i], base + x0, full, g.W - x0);
            } else {
                iv[j][i].zero();
            }
        }
    }
    auto store_q0 = [&](T *plane, int y, const float *v) {
        T *row = plane + (int64_t)y * Qrs + x0;
        if (full) {
            stv<PX>(row, v);
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j)
                if (x0 + j < g.W) st1(row + j, v[j]);
        }
    };
    // with EPI, e = q + gain (p - q) from channel c's row of p, then the store
    auto store_q = [&](int c, int y, float *v) {
        if constexpr (EPI) {
            Row pr;
            ld_row<T, PX>(pr, P + (int64_t)c * Pps + (int64_t)y * Prs + x0, full, g.W - x0);
#pragma unroll
            for (int j = 0; j < PX; ++j) v[j] = lerp(v[j], pr.at(j), gain);
        }
        store_q0(Q + (int64_t)c * Qps, y, v);
    };
    // q = ((mean_b + a_0 I_0) + a_1 I_1) + a_2 I_2, one rounding per term
    auto combine = [&](const float *a, float b, int i, int j) -> float {
        float q = madd(a[0], iv[0][i].at(j), b);
        q = madd(a[1], iv[1][i].at(j), q);
        return madd(a[2], iv[2][i].at(j), q);
    };

    if constexpr (S == 1) {
        // the maps are full resolution (rows padded to 16 floats)
#pragma unroll 1
        for (int c = 0; c < g.C; ++c) {
            const float *Ma = M + (int64_t)(3 * c) * g.lps, *Mb = M + (int64_t)(3 * g.C + c) * g.lps;
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int64_t o = (int64_t)(yb + i) * g.lrs + x0;
                    const f32x4 a0 = ld4(Ma + o), a1 = ld4(Ma + g.lps + o), a2 = ld4(Ma + 2 * g.lps + o);
                    const f32x4 b = ld4(Mb + o);
                    float out[PX];
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        const float a[3] = {a0[j], a1[j], a2[j]};
                        out[j] = combine(a, b[j], i, j);
                    }
                    store_q(c, yb + i, out);
                }
            }
        }
    } else if constexpr (S == 2 || S == 4 || S == 8) {
        // at s = 8 a wave's rows (and a lane's columns) start at 0 or 4 mod
        // 8: their taps share one base and the weights depend on the phase
        constexpr bool PHASE = S == 8;
        constexpr int NL = PHASE ? 2 : cfloor_u(ROWS - 1, S) - cfloor_u(0, S) + 2;
        constexpr int NC = PHASE ? 2 : cfloor_u(PX - 1, S) - cfloor_u(0, S) + 2;
        const int base_y = floordiv(2 * yb + 1 - S, 2 * S);
        const int base_x = floordiv(2 * x0 + 1 - S, 2 * S);
        int ry[NL], cx[NC];
#pragma unroll
        for (int m = 0; m < NL; ++m) ry[m] = clampi(base_y + m, 0, g.Hl - 1);
#pragma unroll
        for (int m = 0; m < NC; ++m) cx[m] = clampi(base_x + m, 0, g.Wl - 1);
        float wx[PX], wy[ROWS];
#pragma unroll
        for (int j = 0; j < PX; ++j)
            wx[j] = PHASE ? (float)((2 * ((x0 & 7) + j) + 1 - 8) & 15) * (1.0f / 16.0f) : cfrac_u(j, S);
#pragma unroll
        for (int i = 0; i < ROWS; ++i)
            wy[i] = PHASE ? (float)((2 * ((yb & 7) + i) + 1 - 8) & 15) * (1.0f / 16.0f) : cfrac_u(i, S);
        if constexpr (S != 8) {
            // q = ((mean_b + a_0 I_0) + a_1 I_1) + a_2 I_2 built map by map (b
            // first) in one accumulator per pixel: the operations and their
            // order are those of combine(), with one map's low-res values and
            // interpolations live at a time.  Fewer registers (4000x3000 RGB
            // fp32 at s = 4: 143 VGPRs against 184, three waves per SIMD against
            // two): 60.5 -> 55.8 us, fp16 76.0 -> 57.5 us, detail 92.0 -> 80.3
            // us; at s = 8 (115 against 136 VGPRs) it was slower, 54.1 against
            // 52.6 us, so s = 8 forms the four maps' values first.
#pragma unroll 1
            for (int c = 0; c < g.C; ++c) {
                float acc[ROWS][PX];
#pragma unroll
                for (int step = 0; step < 4; ++step) {
                    const int mp = step == 0 ? 3 : step - 1;  // b, a_0, a_1, a_2
                    const float *Mm = M + (int64_t)(mp < 3 ? 3 * c + mp : 3 * g.C + c) * g.lps;
                    float v[NL][NC];
#pragma unroll
                    for (int m = 0; m < NL; ++m) {
#pragma unroll
                        for (int k = 0; k < NC; ++k) v[m][k] = Mm[(int64_t)ry[m] * g.lrs + cx[k]];
                    }
#pragma unroll
                    for (int i = 0; i < ROWS; ++i) {
                        const int m0 = cfloor_u(i, S) - cfloor_u(0, S);
#pragma unroll
                        for (int j = 0; j < PX; ++j) {
                            const int k0 = cfloor_u(j, S) - cfloor_u(0, S);
                            const float h0 = lerp(v[m0][k0], v[m0][k0 + 1], wx[j]);
                            const float h1 = lerp(v[m0 + 1][k0], v[m0 + 1][k0 + 1], wx[j]);
                            const float u = lerp(h0, h1, wy[i]);
                            acc[i][j] = step == 0 ? u : madd(u, iv[mp][i].at(j), acc[i][j]);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < ROWS; ++i) {
                    if (i < nrows) store_q(c, yb + i, acc[i]);
                }
            }
        } else {
#pragma unroll 1
            for (int c = 0; c < g.C; ++c) {
                // low-res values of the four maps (a_0, a_1, a_2, b) under the block
                float v[4][NL][NC];
#pragma unroll
                for (int mp = 0; mp < 4; ++mp) {
                    const float *Mm = M + (int64_t)(mp < 3 ? 3 * c + mp : 3 * g.C + c) * g.lps;
#pragma unroll
                    for (int m = 0; m < NL; ++m) {
#pragma unroll
                        for (int k = 0; k < NC; ++k) v[mp][m][k] = Mm[(int64_t)ry[m] * g.lrs + cx[k]];
                    }
                }
#pragma unroll
                for (int i = 0; i < ROWS; ++i) {
                    if (i < nrows) {
                        const int m0 = PHASE ? 0 : cfloor_u(i, S) - cfloor_u(0, S);
                        float out[PX];
#pragma unroll
                        for (int j = 0; j < PX; ++j) {
                            const int k0 = PHASE ? 0 : cfloor_u(j, S) - cfloor_u(0, S);
                            float u[4];
#pragma unroll
                            for (int mp = 0; mp < 4; ++mp) {
                                const float h0 = lerp(v[mp][m0][k0], v[mp][m0][k0 + 1], wx[j]);
                                const float h1 = lerp(v[mp][m0 + 1][k0], v[mp][m0 + 1][k0 + 1], wx[j]);
                                u[mp] = lerp(h0, h1, wy[i]);
                            }
                            out[j] = combine(u, u[3], i, j);
                        }
                        store_q(c, yb + i, out);
                    }
                }
            }
        }
    } else {
        // any other ratio: taps per pixel and per row at run time
        const int s = g.s, s2 = 2 * s;
        const float inv2s = 1.0f / (float)s2;
        int xa[PX], xb[PX];
        float wx[PX];
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            const int num = 2 * (x0 + j) + 1 - s;
            const int l = floordiv(num, s2);
            wx[j] = (float)(num - s2 * l) * inv2s;
            xa[j] = clampi(l, 0, g.Wl - 1);
            xb[j] = clampi(l + 1, 0, g.Wl - 1);
        }
#pragma unroll 1
        for (int c = 0; c < g.C; ++c) {
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int y = yb + i;
                    const int num = 2 * y + 1 - s;
                    const int l = floordiv(num, s2);
                    const float wyi = (float)(num - s2 * l) * inv2s;
                    const int k0 = clampi(l, 0, g.Hl - 1), k1 = clampi(l + 1, 0, g.Hl - 1);
                    float out[PX];
#pragma unroll
                    for (int j = 0; j < PX; ++j) {
                        float u[4];
#pragma unroll
                        for (int mp = 0; mp < 4; ++mp) {
                            const float *Mm = M + (int64_t)(mp < 3 ? 3 * c + mp : 3 * g.C + c) * g.lps;
                            const float *r0p = Mm + (int64_t)k0 * g.lrs, *r1p = Mm + (int64_t)k1 * g.lrs;
                            u[mp] = lerp(lerp(r0p[xa[j]], r0p[xb[j]], wx[j]), lerp(r1p[xa[j]], r1p[xb[j]], wx[j]),
                                         wyi);
                        }
                        out[j] = combine(u, u[3], i, j);
                    }
                    store_q(c, y, out);
                }
            }
        }
    }
}

}  // namespace dev
}  // namespace gf
