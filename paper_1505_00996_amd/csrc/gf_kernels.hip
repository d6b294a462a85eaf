// HIP kernels of the (fast) guided filter for gfx950 (CDNA4, wave64).
//
// Three kernels carry Algorithm 2 of He & Sun, "Fast Guided Filter":
//   k_coeff  : subsample I and p (step 1) while loading a low-res tile plus an
//              r' halo into LDS, form the window sums of I', I'^2, p', I'p'
//              (step 2), then var, cov (step 3) and a, b of Eqs. 2-3 (step 4).
//              Two variants: a sliding-window walk for small r', a separable
//              row pass + column pass for large r'.
//   k_box    : clip-normalised box mean of the 2C coefficient maps (step 5),
//              with the same two variants.
//   k_output : bilinear upsampling of mean_a, mean_b fused with
//              q = mean_a * I + mean_b against the full-resolution I
//              (steps 6-7).  This is the HBM-bound pass: I is read once and q
//              written once with 16-byte accesses; the low-res maps come
//              through the caches.
// Algorithm 1 is the same three kernels at s = 1, where subsampling and
// upsampling are identities and k_output reads mean_a, mean_b directly.
//
// Numerics: samples and coefficients are FP32; window sums are accumulated
// in FP64 (see the coefficient section) and restarted in every tile, so
// rounding neither cancels in flat windows nor drifts across the image.
#include <hip/hip_runtime.h>

#include "gf_internal.h"

namespace gf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

struct bf16 {
    unsigned short bits;
};

// ---------------------------------------------------------------- storage

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float((unsigned)v.bits << 16); }

// float -> bfloat16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ unsigned short f32_to_bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ bf16 from_f32<bf16>(float v) { return bf16{f32_to_bf16_bits(v)}; }

template <typename T> __device__ __forceinline__ float ld(const T *p) { return to_f32(*p); }

// Four consecutive elements, 16 bytes (fp32) or 8 bytes (16-bit), aligned.
__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4 *)p; }
__device__ __forceinline__ f32x4 ld4(const _Float16 *p) {
    f16x4 h = *(const f16x4 *)p;
    return f32x4{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
}
__device__ __forceinline__ f32x4 ld4(const bf16 *p) {
    u16x4 b = *(const u16x4 *)p;
    return f32x4{__uint_as_float((unsigned)b.x << 16), __uint_as_float((unsigned)b.y << 16),
                 __uint_as_float((unsigned)b.z << 16), __uint_as_float((unsigned)b.w << 16)};
}

// Streaming (non-temporal) stores of four outputs.
__device__ __forceinline__ void st4(float *p, f32x4 v) { __builtin_nontemporal_store(v, (f32x4 *)p); }
__device__ __forceinline__ void st4(_Float16 *p, f32x4 v) {
    f16x4 h = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
    __builtin_nontemporal_store(h, (f16x4 *)p);
}
__device__ __forceinline__ void st4(bf16 *p, f32x4 v) {
    u16x4 b = {f32_to_bf16_bits(v.x), f32_to_bf16_bits(v.y), f32_to_bf16_bits(v.z),
               f32_to_bf16_bits(v.w)};
    __builtin_nontemporal_store(b, (u16x4 *)p);
}
template <typename T> __device__ __forceinline__ void st1(T *p, float v) { *p = from_f32<T>(v); }

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int floordiv(int a, int b) {  // b > 0
    int q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Number of in-image positions of a radius-R window centred at i on an n-axis.
__device__ __forceinline__ int clip_len(int i, int R, int n) {
    return min(n - 1, i + R) - max(0, i - R) + 1;
}

// Workgroups are handed to the 8 XCDs round robin (id mod 8).  Launches use
// a grid that is a multiple of 8 and this map gives XCD k the k-th
// contiguous range of logical tiles (row-major), so tiles that share halo
// rows of the low-res maps share an L2.
__device__ __forceinline__ int xcd_tile(int bid) {
    const int per = (int)gridDim.x >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Algorithm 2 step 1, the sample of the low-res map at (ly, lx), which the
// caller keeps inside [0, Hl) x [0, Wl).  The kind is fixed per launch, so
// the loads carry no data-dependent branch and a batch of them can be in
// flight together:
//   kSubId   s = 1: the image itself;
//   kSubNear nearest: full-res s*ly + floor(s/2), clamped to the image (also
//            bilinear with odd s, whose sample centre falls on a pixel);
//   kSubLin  bilinear with even s: the mean of the two pixels on each side
//            of the low-res centre s*ly + (s-1)/2, taps clamped.
constexpr int kSubId = 0, kSubNear = 1, kSubLin = 2;

template <int K, typename T>
__device__ __forceinline__ float sample(const T *__restrict__ img, int64_t rs, int ly, int lx,
                                        const Geo &g) {
    const int s = g.s;
    if constexpr (K == kSubId) {
        return ld(img + (int64_t)ly * rs + lx);
    } else if constexpr (K == kSubNear) {
        const int y = min(s * ly + (s >> 1), g.H - 1), x = min(s * lx + (s >> 1), g.W - 1);
        return ld(img + (int64_t)y * rs + x);
    } else {
        const int y0 = min(s * ly + (s >> 1) - 1, g.H - 1), y1 = min(s * ly + (s >> 1), g.H - 1);
        const int x0 = min(s * lx + (s >> 1) - 1, g.W - 1), x1 = min(s * lx + (s >> 1), g.W - 1);
        const float v00 = ld(img + (int64_t)y0 * rs + x0), v01 = ld(img + (int64_t)y0 * rs + x1);
        const float v10 = ld(img + (int64_t)y1 * rs + x0), v11 = ld(img + (int64_t)y1 * rs + x1);
        return 0.5f * (0.5f * v00 + 0.5f * v01) + 0.5f * (0.5f * v10 + 0.5f * v11);
    }
}

// Sample at region position (ly, lx) shifted by c, or 0 outside the
// low-res map: the load always reads a clamped, valid address and the
// outside case is a select, not a branch.
template <int K, typename T>
__device__ __forceinline__ float sample_shifted(const T *__restrict__ img, int64_t rs, int ly, int lx,
                                                float c, const Geo &g) {
    const bool in = ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
    const float v = sample<K>(img, rs, clampi(ly, 0, g.Hl - 1), clampi(lx, 0, g.Wl - 1), g);
    return in ? v - c : 0.f;
}

// ------------------------------------------------------- staging helpers
//
// Fill SH x SW row-major LDS regions: thread t takes elements t, t + 256, ...,
// kFillPer of them at a time with every global load of the batch issued
// before the first LDS store, so a lane has up to kFillPer (or 2 kFillPer)
// loads in flight instead of one.
constexpr int kFillPer = 12;

template <class F>
__device__ __forceinline__ void fill_region(float *dst, int SH, int SW, F f) {
    const int n = SH * SW;
    for (int base = 0; base < n; base += kFillPer * kThreads) {
        float v[kFillPer];
#pragma unroll
        for (int b = 0; b < kFillPer; ++b) {  // clamped index: every load is unconditional
            const int e = min(base + b * kThreads + (int)threadIdx.x, n - 1);
            const int ry = e / SW;
            v[b] = f(ry, e - ry * SW);
        }
#pragma unroll
        for (int b = 0; b < kFillPer; ++b) {
            const int e = base + b * kThreads + (int)threadIdx.x;
            if (e < n) dst[e] = v[b];
        }
    }
}

template <class F1, class F2>
__device__ __forceinline__ void fill_region2(float *d1, float *d2, int SH, int SW, F1 f1, F2 f2) {
    const int n = SH * SW;
    for (int base = 0; base < n; base += kFillPer * kThreads) {
        float v1[kFillPer], v2[kFillPer];
#pragma unroll
        for (int b = 0; b < kFillPer; ++b) {  // clamped index: every load is unconditional
            const int e = min(base + b * kThreads + (int)threadIdx.x, n - 1);
            const int ry = e / SW, rx = e - ry * SW;
            v1[b] = f1(ry, rx);
            v2[b] = f2(ry, rx);
        }
#pragma unroll
        for (int b = 0; b < kFillPer; ++b) {
            const int e = base + b * kThreads + (int)threadIdx.x;
            if (e < n) {
                d1[e] = v1[b];
                d2[e] = v2[b];
            }
        }
    }
}

// ------------------------------------------------------- coefficients
//
// Statistics of a window are accumulated in FP64.  mean(I*I) - mean(I)^2 and
// mean(I*p) - mean(I) mean(p) cancel almost completely in flat windows; FP64
// sums (the products of FP32 samples are exact in FP64) leave ~1e-16 of
// rounding there, far below any eps, while FP32 sums leave ~1e-8, which at
// eps = 1e-6 moves a by percent.  On gfx950 an FP64 add or FMA issues at the
// rate of an FP32 one (packed FP32 aside), so this costs no more than
// compensated FP32 pairs and is more accurate.  Samples are also shifted by
// the tile's first sample (cI, cP), which keeps the sums small.
//
// Final step shared by both kernels: n samples, sums Su, Suu, Sv, Suv of
// u = I' - cI, v = p' - cP  ->  a, b of Eqs. 2-3.
__device__ __forceinline__ void coeff_from_sums(int n, double Su, double Suu, double Sv, double Suv,
                                                float cI, float cP, float eps, float &a, float &b) {
    // n^2 var and n^2 cov: the two cancelling differences, taken in FP64
    const double nd = (double)n;
    const float n2var = (float)fmax(nd * Suu - Su * Su, 0.0);
    const float n2cov = (float)(nd * Suv - Su * Sv);
    const float inv_n = 1.0f / (float)n;
    const float var = n2var * inv_n * inv_n;
    const float cov = n2cov * inv_n * inv_n;  // Eq. 2 numerator
    const float mI = cI + (float)Su * inv_n, mp = cP + (float)Sv * inv_n;
    a = cov / (var + eps);  // Eq. 2
    b = mp - a * mI;        // Eq. 3
}

// k_coeff_slide: for small r'.  One workgroup = 4 waves over a tile of 64
// low-res columns x 4*TH rows, for ONE channel of p (blockIdx.y).  The
// (4TH + 2r') x (64 + 2r') region of u and v is staged in LDS; then every
// lane owns one output column and slides the (2r'+1)^2 window down TH rows:
// the row entering the window is added and the row leaving it subtracted,
// tap by tap, into FP64 sums.  No row-sum buffer, one barrier.
template <typename T, int K, int TH>
__global__ __launch_bounds__(kThreads) void k_coeff_slide(const T *__restrict__ I, int64_t Irs,
                                                          const T *__restrict__ P, int64_t Prs,
                                                          int64_t Pps, float *__restrict__ coef,
                                                          Geo g, int ntx, int ntiles) {
    extern __shared__ float lds[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    const int c = blockIdx.y;
    const int R = g.R, SH = 4 * TH + 2 * R, SW = 64 + 2 * R;
    const int ty0 = (tile / ntx) * (4 * TH), tx0 = (tile % ntx) * 64;
    const int oy = ty0 - R, ox = tx0 - R;  // region origin in low-res coordinates
    const T *Pc = P + (int64_t)c * Pps;
    float *sU = lds, *sV = lds + SH * SW;

    const float cI = sample<K>(I, Irs, ty0, tx0, g);
    const float cP = sample<K>(Pc, Prs, ty0, tx0, g);
    fill_region2(
        sU, sV, SH, SW,
        [&](int ry, int rx) { return sample_shifted<K>(I, Irs, oy + ry, ox + rx, cI, g); },
        [&](int ry, int rx) { return sample_shifted<K>(Pc, Prs, oy + ry, ox + rx, cP, g); });
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx = tx0 + lane;
    const int r0 = wave * TH;  // region row of the first window row of this wave's first output
    double Su = 0.0, Suu = 0.0, Sv = 0.0, Suv = 0.0;
    auto row = [&](int ry, double sgn) {
        const float *pu = sU + ry * SW + lane, *pv = sV + ry * SW + lane;
        double su = 0.0, suu = 0.0, sv = 0.0, suv = 0.0;
        for (int k = 0; k <= 2 * R; ++k) {
            const double u = pu[k], v = pv[k];
            su += u;
            suu = __builtin_fma(u, u, suu);
            sv += v;
            suv = __builtin_fma(u, v, suv);
        }
        Su = __builtin_fma(sgn, su, Su);
        Suu = __builtin_fma(sgn, suu, Suu);
        Sv = __builtin_fma(sgn, sv, Sv);
        Suv = __builtin_fma(sgn, suv, Suv);
    };
    for (int k = 0; k <= 2 * R; ++k) row(r0 + k, 1.0);
    const int nx = clip_len(lx, R, g.Wl);
    float *ac = coef + (int64_t)c * g.lps;
    float *bc = coef + (int64_t)(g.C + c) * g.lps;
    for (int t = 0; t < TH; ++t) {
        if (t) {
            row(r0 + t + 2 * R, 1.0);
            row(r0 + t - 1, -1.0);
        }
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl) {
            float a, b;
            coeff_from_sums(clip_len(ly, R, g.Hl) * nx, Su, Suu, Sv, Suv, cI, cP, g.eps, a, b);
            ac[(int64_t)ly * g.lrs + lx] = a;
            bc[(int64_t)ly * g.lrs + lx] = b;
        }
    }
}

// k_coeff_sep: any r'.  One workgroup = one TH x TW tile for ONE channel.
// Row pass: each thread slides a (2r'+1)-wide window over kRun consecutive
// outputs of one region row and writes the FP64 sums of u, u*u, v, u*v to
// LDS.  Column pass: each thread owns one column and LC consecutive output
// rows and slides the sums down.  Used when the (2r'+1)^2 taps per output of
// k_coeff_slide would cost more than the two passes.
template <typename T, int K, int TH, int TW, bool STAGE>
__global__ __launch_bounds__(kThreads) void k_coeff_sep(const T *__restrict__ I, int64_t Irs,
                                                        const T *__restrict__ P, int64_t Prs,
                                                        int64_t Pps, float *__restrict__ coef,
                                                        Geo g, int ntx, int ntiles) {
    extern __shared__ double ldsd[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    constexpr int RUNS = TW / kRun, NG = kThreads / TW, LC = TH / NG;
    static_assert(LC * NG == TH && RUNS * kRun == TW, "tile shape");
    const int c = blockIdx.y;
    const int R = g.R, SH = TH + 2 * R, SW = TW + 2 * R;
    const int ty0 = (tile / ntx) * TH, tx0 = (tile % ntx) * TW;
    const int oy = ty0 - R, ox = tx0 - R;
    const T *Pc = P + (int64_t)c * Pps;
    const int plane = SH * TW;
    double *rs = ldsd;                             // 4 row-sum planes of SH x TW
    float *sU = (float *)(rs + 4 * plane);         // staged u, v (STAGE only)
    float *sV = sU + SH * SW;

    const float cI = sample<K>(I, Irs, ty0, tx0, g);
    const float cP = sample<K>(Pc, Prs, ty0, tx0, g);
    auto gU = [&](int ry, int rx) { return sample_shifted<K>(I, Irs, oy + ry, ox + rx, cI, g); };
    auto gV = [&](int ry, int rx) { return sample_shifted<K>(Pc, Prs, oy + ry, ox + rx, cP, g); };
    if (STAGE) {
        fill_region2(sU, sV, SH, SW, gU, gV);
        __syncthreads();
    }
    for (int it = threadIdx.x; it < SH * RUNS; it += kThreads) {
        const int ry = it / RUNS, j0 = (it % RUNS) * kRun;
        auto tap = [&](int rx, double &u, double &v) {
            if (STAGE) {
                u = sU[ry * SW + rx];
                v = sV[ry * SW + rx];
            } else {
                u = gU(ry, rx);
                v = gV(ry, rx);
            }
        };
        double su = 0.0, suu = 0.0, sv = 0.0, suv = 0.0;
        for (int k = 0; k <= 2 * R; ++k) {
            double u, v;
            tap(j0 + k, u, v);
            su += u;
            suu = __builtin_fma(u, u, suu);
            sv += v;
            suv = __builtin_fma(u, v, suv);
        }
        double *o = rs + ry * TW + j0;
        o[0] = su;
        o[plane] = suu;
        o[2 * plane] = sv;
        o[3 * plane] = suv;
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            double ui, vi, uo, vo;
            tap(j0 + t + 2 * R, ui, vi);
            tap(j0 + t - 1, uo, vo);
            su += ui - uo;
            suu += __builtin_fma(ui, ui, -uo * uo);
            sv += vi - vo;
            suv += __builtin_fma(ui, vi, -uo * vo);
            o[t] = su;
            o[t + plane] = suu;
            o[t + 2 * plane] = sv;
            o[t + 3 * plane] = suv;
        }
    }
    __syncthreads();

    const int col = threadIdx.x % TW, r0 = (threadIdx.x / TW) * LC;
    const int lx = tx0 + col;
    const int nx = clip_len(lx, R, g.Wl);
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k <= 2 * R; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) S[m] += rs[(r0 + k) * TW + col + m * plane];
    float *ac = coef + (int64_t)c * g.lps;
    float *bc = coef + (int64_t)(g.C + c) * g.lps;
#pragma unroll
    for (int t = 0; t < LC; ++t) {
        if (t) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
                S[m] += rs[(r0 + t + 2 * R) * TW + col + m * plane] - rs[(r0 + t - 1) * TW + col + m * plane];
        }
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl) {
            float a, b;
            coeff_from_sums(clip_len(ly, R, g.Hl) * nx, S[0], S[1], S[2], S[3], cI, cP, g.eps, a, b);
            ac[(int64_t)ly * g.lrs + lx] = a;
            bc[(int64_t)ly * g.lrs + lx] = b;
        }
    }
}

// ---------------------------------------------------------------- box means
//
// Clip-normalised box mean of one low-res FP32 plane per blockIdx.y (the
// coefficient maps a_c, b_c: Algorithm 2 step 5).  FP64 sums.

// k_box_slide: small r'; same tiling and window walk as k_coeff_slide.
template <int TH>
__global__ __launch_bounds__(kThreads) void k_box_slide(const float *__restrict__ src,
                                                        float *__restrict__ dst, Geo g, int ntx,
                                                        int ntiles) {
    extern __shared__ float lds[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    const int R = g.R, SH = 4 * TH + 2 * R, SW = 64 + 2 * R;
    const int ty0 = (tile / ntx) * (4 * TH), tx0 = (tile % ntx) * 64;
    const int oy = ty0 - R, ox = tx0 - R;
    const float *S = src + (int64_t)blockIdx.y * g.lps;
    float *D = dst + (int64_t)blockIdx.y * g.lps;
    float *sX = lds;
    fill_region(sX, SH, SW, [&](int ry, int rx) -> float {
        const int ly = oy + ry, lx = ox + rx;
        const bool in = ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
        const float v = S[(int64_t)clampi(ly, 0, g.Hl - 1) * g.lrs + clampi(lx, 0, g.Wl - 1)];
        return in ? v : 0.f;
    });
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx = tx0 + lane, r0 = wave * TH;
    double A = 0.0;
    auto row = [&](int ry, double sgn) {
        const float *px = sX + ry * SW + lane;
        double sx = 0.0;
        for (int k = 0; k <= 2 * R; ++k) sx += px[k];
        A = __builtin_fma(sgn, sx, A);
    };
    for (int k = 0; k <= 2 * R; ++k) row(r0 + k, 1.0);
    const int nx = clip_len(lx, R, g.Wl);
    for (int t = 0; t < TH; ++t) {
        if (t) {
            row(r0 + t + 2 * R, 1.0);
            row(r0 + t - 1, -1.0);
        }
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl) D[(int64_t)ly * g.lrs + lx] = (float)(A / (double)(clip_len(ly, R, g.Hl) * nx));
    }
}

// k_box_sep: any r'; row pass into LDS (FP64 sums), column pass in registers.
template <int TH, bool STAGE>
__global__ __launch_bounds__(kThreads) void k_box_sep(const float *__restrict__ src,
                                                      float *__restrict__ dst, Geo g, int ntx,
                                                      int ntiles) {
    extern __shared__ double ldsd[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    constexpr int TW = kTileW, RUNS = TW / kRun, NG = kThreads / TW, LC = TH / NG;
    const int R = g.R, SH = TH + 2 * R, SW = TW + 2 * R;
    const int ty0 = (tile / ntx) * TH, tx0 = (tile % ntx) * TW;
    const int oy = ty0 - R, ox = tx0 - R;
    const float *S = src + (int64_t)blockIdx.y * g.lps;
    float *D = dst + (int64_t)blockIdx.y * g.lps;
    double *rA = ldsd;
    float *sX = (float *)(rA + SH * TW);
    auto gX = [&](int ry, int rx) -> float {
        const int ly = oy + ry, lx = ox + rx;
        const bool in = ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
        const float v = S[(int64_t)clampi(ly, 0, g.Hl - 1) * g.lrs + clampi(lx, 0, g.Wl - 1)];
        return in ? v : 0.f;
    };
    if (STAGE) {
        fill_region(sX, SH, SW, gX);
        __syncthreads();
    }
    for (int it = threadIdx.x; it < SH * RUNS; it += kThreads) {
        const int ry = it / RUNS, j0 = (it % RUNS) * kRun;
        auto x = [&](int rx) -> double { return STAGE ? sX[ry * SW + rx] : gX(ry, rx); };
        double A = 0.0;
        for (int k = 0; k <= 2 * R; ++k) A += x(j0 + k);
        double *oa = rA + ry * TW + j0;
        oa[0] = A;
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            A += x(j0 + t + 2 * R) - x(j0 + t - 1);
            oa[t] = A;
        }
    }
    __syncthreads();
    const int col = threadIdx.x % TW, r0 = (threadIdx.x / TW) * LC;
    const int lx = tx0 + col;
    const int nx = clip_len(lx, R, g.Wl);
    double A = 0.0;
    for (int k = 0; k <= 2 * R; ++k) A += rA[(r0 + k) * TW + col];
#pragma unroll
    for (int t = 0; t < LC; ++t) {
        if (t) A += rA[(r0 + t + 2 * R) * TW + col] - rA[(r0 + t - 1) * TW + col];
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl) D[(int64_t)ly * g.lrs + lx] = (float)(A / (double)(clip_len(ly, R, g.Hl) * nx));
    }
}

// ---------------------------------------------------------------- k_output
//
// One workgroup = 4 waves; a wave covers 256 full-res columns (4 per lane)
// and ROWS = 8 consecutive rows starting at a multiple of 8.  A lane first
// loads its 8 x 4 guide pixels (all loads in flight together); then, channel
// by channel, it loads the low-res rows and columns of mean_a, mean_b that
// its pixels interpolate from, interpolates them horizontally once, and for
// every row finishes the bilinear weights and writes q = a*I + b with
// non-temporal 16-byte stores.
//
// Upsampling geometry (half-pixel centres): full-res x maps to low-res
// u = (x + 0.5)/s - 0.5 = (2x + 1 - s) / (2s), taps floor(u), floor(u) + 1
// clamped to the map.  For s in {2, 4, 8}, lanes start at x0 = 0 mod 4 and
// waves at y = 0 mod 8, so which low-res rows/columns each pixel uses,
// relative to the first one, is known at compile time.

// floor((2x + 1 - s) / (2s)) for compile-time use
constexpr int cfloor_u(int x, int s) {
    return (2 * x + 1 - s) >= 0 ? (2 * x + 1 - s) / (2 * s) : -((2 * s - 1 - (2 * x + 1 - s)) / (2 * s));
}
constexpr float cfrac_u(int x, int s) {
    return (float)((2 * x + 1 - s) - 2 * s * cfloor_u(x, s)) / (float)(2 * s);
}

template <typename T, int CC, int S, int ROWS>
__global__ __launch_bounds__(kThreads) void k_output(const T *__restrict__ I, int64_t Irs,
                                                     T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                     const float *__restrict__ M, Geo g, int c0,
                                                     int ntx, int ntiles, int vec) {
    static_assert(ROWS == 8, "row patterns assume waves start at multiples of 8");
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = (tile % ntx) * kOutTileW + lane * kOutPx;
    const int yb = (tile / ntx) * (4 * ROWS) + wave * ROWS;
    const int nrows = min(ROWS, g.H - yb);
    if (x0 >= g.W || nrows <= 0) return;  // no barriers below
    const bool full = vec && (x0 + 3 < g.W);

    f32x4 iv[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        iv[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (i < nrows) {
            const T *row = I + (int64_t)(yb + i) * Irs + x0;
            if (full) {
                iv[i] = ld4(row);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (x0 + j < g.W) iv[i][j] = ld(row + j);
            }
        }
    }
    auto store_q = [&](T *plane, int y, f32x4 v) {
        T *row = plane + (int64_t)y * Qrs + x0;
        if (full) {
            st4(row, v);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < g.W) st1(row + j, v[j]);
        }
    };

    if constexpr (S == 1) {
        // Algorithm 1: the maps are full resolution; rows are padded to a
        // multiple of 16 floats, so the 16-byte read at x0 stays in the row.
#pragma unroll 1
        for (int c = 0; c < CC; ++c) {
            const float *Ma = M + (int64_t)(c0 + c) * g.lps;
            const float *Mb = M + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * Qps;
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int y = yb + i;
                    const f32x4 a = ld4(Ma + (int64_t)y * g.lrs + x0);
                    const f32x4 b = ld4(Mb + (int64_t)y * g.lrs + x0);
                    store_q(Qc, y, a * iv[i] + b);
                }
            }
        }
    } else if constexpr (S == 2 || S == 4 || S == 8) {
        // low-res rows base_y .. base_y + NL - 1 and columns base_x .. base_x + NC - 1
        constexpr int NL = cfloor_u(ROWS - 1, S) - cfloor_u(0, S) + 2;
        constexpr int NC = cfloor_u(3, S) - cfloor_u(0, S) + 2;
        const int base_y = floordiv(2 * yb + 1 - S, 2 * S);
        const int base_x = floordiv(2 * x0 + 1 - S, 2 * S);
        int ry[NL], cx[NC];
#pragma unroll
        for (int m = 0; m < NL; ++m) ry[m] = clampi(base_y + m, 0, g.Hl - 1);
#pragma unroll
        for (int m = 0; m < NC; ++m) cx[m] = clampi(base_x + m, 0, g.Wl - 1);
        // horizontal weights: compile time when s divides 4; for s = 8 they
        // depend on whether the lane starts at 0 or 4 mod 8
        float wx[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            wx[j] = (S == 8) ? (float)((2 * ((x0 & 7) + j) + 1 - 8) & 15) * (1.0f / 16.0f)
                             : cfrac_u(j, S);
#pragma unroll 1
        for (int c = 0; c < CC; ++c) {
            const float *Ma = M + (int64_t)(c0 + c) * g.lps;
            const float *Mb = M + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * Qps;
            float ha[NL][4], hb[NL][4];
#pragma unroll
            for (int m = 0; m < NL; ++m) {
                const float *ra = Ma + (int64_t)ry[m] * g.lrs;
                const float *rb = Mb + (int64_t)ry[m] * g.lrs;
                float va[NC], vb[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    va[k] = ra[cx[k]];
                    vb[k] = rb[cx[k]];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k0 = cfloor_u(j, S) - cfloor_u(0, S);  // 0 for s = 8 as well
                    ha[m][j] = va[k0] + wx[j] * (va[k0 + 1] - va[k0]);
                    hb[m][j] = vb[k0] + wx[j] * (vb[k0 + 1] - vb[k0]);
                }
            }
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int m0 = cfloor_u(i, S) - cfloor_u(0, S);
                    const float wy = cfrac_u(i, S);
                    f32x4 out;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float a = ha[m0][j] + wy * (ha[m0 + 1][j] - ha[m0][j]);
                        const float b = hb[m0][j] + wy * (hb[m0 + 1][j] - hb[m0][j]);
                        out[j] = a * iv[i][j] + b;
                    }
                    store_q(Qc, yb + i, out);
                }
            }
        }
    } else {
        // any other ratio: taps computed per pixel and per row at run time
        const int s = g.s, s2 = 2 * s;
        const float inv2s = 1.0f / (float)s2;
        int xa[4], xb[4];
        float wx[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int num = 2 * (x0 + j) + 1 - s;
            const int l = floordiv(num, s2);
            wx[j] = (float)(num - s2 * l) * inv2s;
            xa[j] = clampi(l, 0, g.Wl - 1);
            xb[j] = clampi(l + 1, 0, g.Wl - 1);
        }
#pragma unroll 1
        for (int c = 0; c < CC; ++c) {
            const float *Ma = M + (int64_t)(c0 + c) * g.lps;
            const float *Mb = M + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * Qps;
#pragma unroll 1
            for (int i = 0; i < nrows; ++i) {
                const int y = yb + i;
                const int num = 2 * y + 1 - s;
                const int l = floordiv(num, s2);
                const float wy = (float)(num - s2 * l) * inv2s;
                const int k0 = clampi(l, 0, g.Hl - 1), k1 = clampi(l + 1, 0, g.Hl - 1);
                const float *ra0 = Ma + (int64_t)k0 * g.lrs, *ra1 = Ma + (int64_t)k1 * g.lrs;
                const float *rb0 = Mb + (int64_t)k0 * g.lrs, *rb1 = Mb + (int64_t)k1 * g.lrs;
                f32x4 iy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    if (r == i) iy = iv[r];
                f32x4 out;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float a0 = ra0[xa[j]] + wx[j] * (ra0[xb[j]] - ra0[xa[j]]);
                    const float a1 = ra1[xa[j]] + wx[j] * (ra1[xb[j]] - ra1[xa[j]]);
                    const float b0 = rb0[xa[j]] + wx[j] * (rb0[xb[j]] - rb0[xa[j]]);
                    const float b1 = rb1[xa[j]] + wx[j] * (rb1[xb[j]] - rb1[xa[j]]);
                    out[j] = (a0 + wy * (a1 - a0)) * iy[j] + (b0 + wy * (b1 - b0));
                }
                store_q(Qc, y, out);
            }
        }
    }
}

// ---------------------------------------------------------------- launch

int grid8(int n) { return ((n + 7) / 8) * 8; }

// Dynamic LDS above 64 KB has to be allowed per kernel (gfx950 has 160 KB).
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

template <typename T, int K>
hipError_t coeff_tk(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                    hipStream_t st) {
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
    const dim3 block(kThreads);
    const size_t lds = coeff_lds_bytes(t, g.R);
    if (t.coeff_slide) {
        const int ntx = (g.Wl + 63) / 64, nty = (g.Hl + 4 * t.coeff_th - 1) / (4 * t.coeff_th);
        const int ntiles = ntx * nty;
        const dim3 grid(grid8(ntiles), g.C);
#define GF_SLIDE(TH)                                                                               \
    {                                                                                              \
        allow_lds(k_coeff_slide<T, K, TH>, lds);                                                   \
        hipLaunchKernelGGL((k_coeff_slide<T, K, TH>), grid, block, lds, st, Ip, I.rs, Pp, P.rs, P.ps, \
                           coef, g, ntx, ntiles);                                                  \
    }
        if (t.coeff_th == 4) GF_SLIDE(4) else if (t.coeff_th == 8) GF_SLIDE(8) else GF_SLIDE(16)
#undef GF_SLIDE
        return hipGetLastError();
    }
    const int ntx = (g.Wl + t.coeff_tw - 1) / t.coeff_tw;
    const int nty = (g.Hl + t.coeff_th - 1) / t.coeff_th;
    const int ntiles = ntx * nty;
    const dim3 grid(grid8(ntiles), g.C);
#define GF_SEP(TH, TW, STG)                                                                           \
    {                                                                                                 \
        allow_lds(k_coeff_sep<T, K, TH, TW, STG>, lds);                                               \
        hipLaunchKernelGGL((k_coeff_sep<T, K, TH, TW, STG>), grid, block, lds, st, Ip, I.rs, Pp, P.rs, \
                           P.ps, coef, g, ntx, ntiles);                                               \
    }
    if (!t.coeff_stage) {
        if (t.coeff_th == 8) GF_SEP(8, 32, false) else GF_SEP(16, 32, false)
    } else if (t.coeff_th == 32) {
        if (t.coeff_tw == 64) GF_SEP(32, 64, true) else GF_SEP(32, 32, true)
    } else {
        if (t.coeff_tw == 64) GF_SEP(16, 64, true) else GF_SEP(16, 32, true)
    }
#undef GF_SEP
    return hipGetLastError();
}

template <typename T>
hipError_t coeff_t(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                   hipStream_t st) {
    if (g.s == 1) return coeff_tk<T, kSubId>(I, P, coef, g, t, st);
    if (g.sub == GF_SUB_NEAREST || (g.s & 1)) return coeff_tk<T, kSubNear>(I, P, coef, g, t, st);
    return coeff_tk<T, kSubLin>(I, P, coef, g, t, st);
}

template <typename T, int CC>
hipError_t output_cc(const View &I, const View &Q, const float *mean, const Geo &g, int c0,
                     const TileCfg &t, bool vec, hipStream_t st) {
    constexpr int ROWS = 8;
    const int ntx = (g.W + kOutTileW - 1) / kOutTileW;
    const int nty = (g.H + 4 * ROWS - 1) / (4 * ROWS);
    const int ntiles = ntx * nty;
    const T *Ip = (const T *)I.data;
    T *Qp = (T *)Q.data + (int64_t)c0 * Q.ps;
    const dim3 grid(grid8(ntiles)), block(kThreads);
    (void)t;
#define GF_OUT(SS)                                                                               \
    hipLaunchKernelGGL((k_output<T, CC, SS, ROWS>), grid, block, 0, st, Ip, I.rs, Qp, Q.rs, Q.ps, \
                       mean, g, c0, ntx, ntiles, (int)vec)
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

template <typename T>
hipError_t output_t(const View &I, const View &Q, const float *mean, const Geo &g,
                    const TileCfg &t, bool vec, hipStream_t st) {
    for (int c0 = 0; c0 < g.C; c0 += 3) {
        const int cc = g.C - c0 < 3 ? g.C - c0 : 3;
        hipError_t e = cc == 3 ? output_cc<T, 3>(I, Q, mean, g, c0, t, vec, st)
                     : cc == 2 ? output_cc<T, 2>(I, Q, mean, g, c0, t, vec, st)
                               : output_cc<T, 1>(I, Q, mean, g, c0, t, vec, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_coeff(gf_dtype dt, const View &I, const View &P, float *coef, const Geo &g,
                        const TileCfg &t, hipStream_t st) {
    switch (dt) {
        case GF_F32: return coeff_t<float>(I, P, coef, g, t, st);
        case GF_F16: return coeff_t<_Float16>(I, P, coef, g, t, st);
        case GF_BF16: return coeff_t<bf16>(I, P, coef, g, t, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_box(const float *src, float *dst, const Geo &g, const TileCfg &t, hipStream_t st) {
    const size_t lds = box_lds_bytes(t, g.R);
    const dim3 block(kThreads);
    if (t.box_slide) {
        const int ntx = (g.Wl + 63) / 64, nty = (g.Hl + 4 * t.box_th - 1) / (4 * t.box_th);
        const int ntiles = ntx * nty;
        const dim3 grid(grid8(ntiles), 2 * g.C);
#define GF_BSLIDE(TH)                                                                        \
    {                                                                                        \
        allow_lds(k_box_slide<TH>, lds);                                                     \
        hipLaunchKernelGGL((k_box_slide<TH>), grid, block, lds, st, src, dst, g, ntx, ntiles); \
    }
        if (t.box_th == 4) GF_BSLIDE(4) else if (t.box_th == 8) GF_BSLIDE(8) else GF_BSLIDE(16)
#undef GF_BSLIDE
        return hipGetLastError();
    }
    const int ntx = (g.Wl + kTileW - 1) / kTileW;
    const int nty = (g.Hl + t.box_th - 1) / t.box_th;
    const int ntiles = ntx * nty;
    const dim3 grid(grid8(ntiles), 2 * g.C);
#define GF_BOX(TH, STG)                                                                        \
    {                                                                                          \
        allow_lds(k_box_sep<TH, STG>, lds);                                                    \
        hipLaunchKernelGGL((k_box_sep<TH, STG>), grid, block, lds, st, src, dst, g, ntx, ntiles); \
    }
    if (t.box_th == 32) {
        if (t.box_stage) GF_BOX(32, true) else GF_BOX(32, false)
    } else if (t.box_th == 16) {
        if (t.box_stage) GF_BOX(16, true) else GF_BOX(16, false)
    } else {
        if (t.box_stage) GF_BOX(8, true) else GF_BOX(8, false)
    }
#undef GF_BOX
    return hipGetLastError();
}

hipError_t launch_output(gf_dtype dt, const View &I, const View &Q, const float *mean,
                         const Geo &g, const TileCfg &t, bool vec, hipStream_t st) {
    switch (dt) {
        case GF_F32: return output_t<float>(I, Q, mean, g, t, vec, st);
        case GF_F16: return output_t<_Float16>(I, Q, mean, g, t, vec, st);
        case GF_BF16: return output_t<bf16>(I, Q, mean, g, t, vec, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace gf
