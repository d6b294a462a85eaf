// HIP kernels of the (fast) guided filter for gfx950 (CDNA4, wave64).
//
// Three kernels carry Algorithm 2 of He & Sun, "Fast Guided Filter":
//   k_coeff  : subsample I and p (step 1) while loading a low-res tile plus an
//              r' halo, form the window sums of I', I'^2, p', I'p' with a
//              separable row pass (LDS) and column pass (registers) (step 2),
//              then var, cov (step 3) and a, b of Eqs. 2-3 (step 4).
//   k_box    : clip-normalised box mean of the 2C coefficient maps (step 5).
//   k_output : bilinear upsampling of mean_a, mean_b fused with
//              q = mean_a * I + mean_b against the full-resolution I
//              (steps 6-7).  This is the HBM-bound pass: I is read once and q
//              written once with 16-byte accesses; the low-res maps come
//              through the caches.
// Algorithm 1 is the same three kernels at s = 1, where subsampling and
// upsampling are identities and k_output reads mean_a, mean_b directly.
//
// Numerics: window sums are FP32.  Each k_coeff tile subtracts a reference
// value (its first low-res sample of I and of each p channel) before
// summing, so var = E[(I-c)^2] - E[I-c]^2 does not cancel two numbers near
// mean(I)^2; sums are restarted every tile and slide over at most kRun
// outputs, so rounding does not drift across the image.
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

// Algorithm 2 step 1 at low-res pixel (ly, lx): nearest takes full-res
// s*ly + floor(s/2); bilinear with even s averages the two pixels around the
// low-res centre s*ly + (s-1)/2 on each axis; taps clamp to the image.
template <typename T>
__device__ __forceinline__ float subsample_at(const T *__restrict__ img, int64_t rs, int ly, int lx,
                                              const Geo &g) {
    const int s = g.s;
    if (s == 1) return ld(img + (int64_t)ly * rs + lx);
    if (g.sub == GF_SUB_NEAREST || (s & 1)) {
        const int y = min(s * ly + (s >> 1), g.H - 1), x = min(s * lx + (s >> 1), g.W - 1);
        return ld(img + (int64_t)y * rs + x);
    }
    const int y0 = min(s * ly + (s >> 1) - 1, g.H - 1), y1 = min(s * ly + (s >> 1), g.H - 1);
    const int x0 = min(s * lx + (s >> 1) - 1, g.W - 1), x1 = min(s * lx + (s >> 1), g.W - 1);
    const float v00 = ld(img + (int64_t)y0 * rs + x0), v01 = ld(img + (int64_t)y0 * rs + x1);
    const float v10 = ld(img + (int64_t)y1 * rs + x0), v11 = ld(img + (int64_t)y1 * rs + x1);
    return 0.5f * (0.5f * v00 + 0.5f * v01) + 0.5f * (0.5f * v10 + 0.5f * v11);
}

// ------------------------------------------------------- window-sum passes
//
// A tile produces TH x kTileW low-res outputs from a region of
// (TH + 2R) x (kTileW + 2R) samples.  The row pass writes, for every region
// row, the horizontal window sums of two derived maps into LDS (rA, rB); each
// thread owns kRun consecutive outputs of one row and slides its window.
// The column pass gives every thread one column and TH/4 consecutive rows.

// Row pass.  fu(ry, rx), fv(ry, rx) return region samples.  PAIR = false:
// rA = sum u, rB = sum u*u.  PAIR = true: rA = sum v, rB = sum u*v.
template <bool PAIR, class FU, class FV>
__device__ __forceinline__ void row_pass(FU fu, FV fv, float *rA, float *rB, int SH, int R) {
    constexpr int runs = kTileW / kRun;
    for (int it = threadIdx.x; it < SH * runs; it += kThreads) {
        const int ry = it / runs, j0 = (it % runs) * kRun;
        float A = 0.f, B = 0.f;
        for (int k = 0; k <= 2 * R; ++k) {
            const float u = fu(ry, j0 + k);
            if (PAIR) {
                const float v = fv(ry, j0 + k);
                A += v;
                B += u * v;
            } else {
                A += u;
                B += u * u;
            }
        }
        float *oa = rA + ry * kTileW + j0, *ob = rB + ry * kTileW + j0;
        oa[0] = A;
        ob[0] = B;
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            const float ui = fu(ry, j0 + t + 2 * R), uo = fu(ry, j0 + t - 1);
            if (PAIR) {
                const float vi = fv(ry, j0 + t + 2 * R), vo = fv(ry, j0 + t - 1);
                A += vi - vo;
                B += ui * vi - uo * vo;
            } else {
                A += ui - uo;
                B += ui * ui - uo * uo;
            }
            oa[t] = A;
            ob[t] = B;
        }
    }
}

// Single-map row pass: rA = sum x.
template <class FX>
__device__ __forceinline__ void row_pass1(FX fx, float *rA, int SH, int R) {
    constexpr int runs = kTileW / kRun;
    for (int it = threadIdx.x; it < SH * runs; it += kThreads) {
        const int ry = it / runs, j0 = (it % runs) * kRun;
        float A = 0.f;
        for (int k = 0; k <= 2 * R; ++k) A += fx(ry, j0 + k);
        float *oa = rA + ry * kTileW + j0;
        oa[0] = A;
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            A += fx(ry, j0 + t + 2 * R) - fx(ry, j0 + t - 1);
            oa[t] = A;
        }
    }
}

// ---------------------------------------------------------------- k_coeff
//
// One workgroup = one low-res tile of TH x 64 outputs.  LDS holds the
// mean-shifted samples of I' and of one channel of p' (when STAGE), and the
// two row-sum buffers.  Channels of p are processed one after the other;
// mean(I) and 1/(var+eps) stay in registers across them.
template <typename T, int TH, bool STAGE>
__global__ __launch_bounds__(kThreads) void k_coeff(const T *__restrict__ I, int64_t Irs,
                                                    const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                                    float *__restrict__ coef, Geo g, int ntx,
                                                    int ntiles) {
    extern __shared__ float lds[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;  // uniform per workgroup: no barrier is skipped by part of it
    constexpr int LC = TH / 4;   // rows per thread in the column pass
    const int R = g.R, SH = TH + 2 * R, SW = kTileW + 2 * R;
    const int ty0 = (tile / ntx) * TH, tx0 = (tile % ntx) * kTileW;
    const int oy = ty0 - R, ox = tx0 - R;  // region origin in low-res coordinates

    float *sI = lds;
    float *sP = STAGE ? sI + SH * SW : nullptr;
    float *rA = STAGE ? sP + SH * SW : lds;
    float *rB = rA + SH * kTileW;

    // Mean-shift references: the samples at the tile's first output.
    const float cI = subsample_at(I, Irs, ty0, tx0, g);

    auto inside = [&](int ry, int rx) {
        const int ly = oy + ry, lx = ox + rx;
        return ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
    };
    auto gI = [&](int ry, int rx) -> float {
        return inside(ry, rx) ? subsample_at(I, Irs, oy + ry, ox + rx, g) - cI : 0.f;
    };
    auto fill = [&](float *dst, const T *src, int64_t rs, float c) {
        for (int e = threadIdx.x; e < SH * SW; e += kThreads) {
            const int ry = e / SW, rx = e - ry * SW;
            dst[e] = inside(ry, rx) ? subsample_at(src, rs, oy + ry, ox + rx, g) - c : 0.f;
        }
    };

    const int col = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * LC;
    const int lx = tx0 + col;
    const int nx = clip_len(lx, R, g.Wl);

    // mean(I) and 1 / (var(I) + eps) for this thread's outputs
    float mI[LC], inv[LC];
    if (STAGE) {
        fill(sI, I, Irs, cI);
        __syncthreads();
        row_pass<false>([&](int y, int x) { return sI[y * SW + x]; }, [](int, int) { return 0.f; },
                        rA, rB, SH, R);
    } else {
        row_pass<false>(gI, [](int, int) { return 0.f; }, rA, rB, SH, R);
    }
    __syncthreads();
    {
        float A = 0.f, B = 0.f;
        for (int k = 0; k <= 2 * R; ++k) {
            A += rA[(r0 + k) * kTileW + col];
            B += rB[(r0 + k) * kTileW + col];
        }
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            if (t) {
                A += rA[(r0 + t + 2 * R) * kTileW + col] - rA[(r0 + t - 1) * kTileW + col];
                B += rB[(r0 + t + 2 * R) * kTileW + col] - rB[(r0 + t - 1) * kTileW + col];
            }
            const int n = max(1, clip_len(ty0 + r0 + t, R, g.Hl) * nx);
            const float invn = 1.0f / (float)n;
            const float m = A * invn;
            const float var = fmaxf(B * invn - m * m, 0.f);
            mI[t] = m;
            inv[t] = 1.0f / (var + g.eps);
        }
    }
    __syncthreads();

    for (int c = 0; c < g.C; ++c) {
        const T *Pc = P + (int64_t)c * Pps;
        const float cP = subsample_at(Pc, Prs, ty0, tx0, g);
        if (STAGE) {
            fill(sP, Pc, Prs, cP);
            __syncthreads();
            row_pass<true>([&](int y, int x) { return sI[y * SW + x]; },
                           [&](int y, int x) { return sP[y * SW + x]; }, rA, rB, SH, R);
        } else {
            row_pass<true>(gI,
                           [&](int ry, int rx) -> float {
                               return inside(ry, rx) ? subsample_at(Pc, Prs, oy + ry, ox + rx, g) - cP
                                                     : 0.f;
                           },
                           rA, rB, SH, R);
        }
        __syncthreads();
        float A = 0.f, B = 0.f;
        for (int k = 0; k <= 2 * R; ++k) {
            A += rA[(r0 + k) * kTileW + col];
            B += rB[(r0 + k) * kTileW + col];
        }
        float *ac = coef + (int64_t)c * g.lps;
        float *bc = coef + (int64_t)(g.C + c) * g.lps;
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            if (t) {
                A += rA[(r0 + t + 2 * R) * kTileW + col] - rA[(r0 + t - 1) * kTileW + col];
                B += rB[(r0 + t + 2 * R) * kTileW + col] - rB[(r0 + t - 1) * kTileW + col];
            }
            const int ly = ty0 + r0 + t;
            if (ly < g.Hl && lx < g.Wl) {
                const int n = clip_len(ly, R, g.Hl) * nx;
                const float invn = 1.0f / (float)n;
                const float mp = A * invn;                   // mean of p - cP
                const float cov = B * invn - mI[t] * mp;     // Eq. 2 numerator
                const float a = cov * inv[t];                // Eq. 2
                const float b = (cP + mp) - a * (cI + mI[t]);  // Eq. 3
                ac[(int64_t)ly * g.lrs + lx] = a;
                bc[(int64_t)ly * g.lrs + lx] = b;
            }
        }
        __syncthreads();  // rA/rB (and sP) are rewritten by the next channel
    }
}

// ---------------------------------------------------------------- k_box
//
// Clip-normalised box mean of one low-res FP32 plane per blockIdx.y.
template <int TH, bool STAGE>
__global__ __launch_bounds__(kThreads) void k_box(const float *__restrict__ src,
                                                  float *__restrict__ dst, Geo g, int ntx,
                                                  int ntiles) {
    extern __shared__ float lds[];
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    constexpr int LC = TH / 4;
    const int R = g.R, SH = TH + 2 * R, SW = kTileW + 2 * R;
    const int ty0 = (tile / ntx) * TH, tx0 = (tile % ntx) * kTileW;
    const int oy = ty0 - R, ox = tx0 - R;
    const float *S = src + (int64_t)blockIdx.y * g.lps;
    float *D = dst + (int64_t)blockIdx.y * g.lps;

    float *sX = lds;
    float *rA = STAGE ? sX + SH * SW : lds;
    auto gX = [&](int ry, int rx) -> float {
        const int ly = oy + ry, lx = ox + rx;
        return (ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl) ? S[(int64_t)ly * g.lrs + lx] : 0.f;
    };
    if (STAGE) {
        for (int e = threadIdx.x; e < SH * SW; e += kThreads) {
            const int ry = e / SW, rx = e - ry * SW;
            sX[e] = gX(ry, rx);
        }
        __syncthreads();
        row_pass1([&](int y, int x) { return sX[y * SW + x]; }, rA, SH, R);
    } else {
        row_pass1(gX, rA, SH, R);
    }
    __syncthreads();

    const int col = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * LC;
    const int lx = tx0 + col;
    const int nx = clip_len(lx, R, g.Wl);
    float A = 0.f;
    for (int k = 0; k <= 2 * R; ++k) A += rA[(r0 + k) * kTileW + col];
#pragma unroll
    for (int t = 0; t < LC; ++t) {
        if (t) A += rA[(r0 + t + 2 * R) * kTileW + col] - rA[(r0 + t - 1) * kTileW + col];
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl) {
            const int n = clip_len(ly, R, g.Hl) * nx;
            D[(int64_t)ly * g.lrs + lx] = A / (float)n;
        }
    }
}

// ---------------------------------------------------------------- k_output
//
// One workgroup = 4 waves; a wave covers 256 full-res columns (4 per lane)
// and `rows` consecutive rows.  Each lane computes its horizontal taps and
// weights once, keeps the horizontally interpolated mean_a, mean_b of the
// two low-res rows that bracket the current full-res row in registers, and
// reloads them only when the bracket moves (every s rows).  q = a*I + b is
// written with non-temporal 16-byte stores.  CC channels, starting at c0.
// S is the compile-time ratio (0 = read g.s at run time).
template <typename T, int CC, int S>
__global__ __launch_bounds__(kThreads) void k_output(const T *__restrict__ I, int64_t Irs,
                                                     T *__restrict__ Q, int64_t Qrs, int64_t Qps,
                                                     const float *__restrict__ M, Geo g, int c0,
                                                     int ntx, int ntiles, int rows, int vec) {
    const int tile = xcd_tile(blockIdx.x);
    if (tile >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = (tile % ntx) * kOutTileW + lane * kOutPx;
    const int yb = (tile / ntx) * (4 * rows) + wave * rows;
    const int ye = min(yb + rows, g.H);
    if (x0 >= g.W || yb >= ye) return;  // no barriers below
    const bool full = vec && (x0 + 3 < g.W);

    const float *Ma[CC], *Mb[CC];
    T *Qc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) {
        Ma[c] = M + (int64_t)(c0 + c) * g.lps;
        Mb[c] = M + (int64_t)(g.C + c0 + c) * g.lps;
        Qc[c] = Q + (int64_t)c * Qps;
    }

    auto load_I = [&](int y) -> f32x4 {
        const T *row = I + (int64_t)y * Irs + x0;
        if (full) return ld4(row);
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (x0 + j < g.W) v[j] = ld(row + j);
        return v;
    };
    auto store_q = [&](int c, int y, f32x4 v) {
        T *row = Qc[c] + (int64_t)y * Qrs + x0;
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
        for (int y = yb; y < ye; ++y) {
            const f32x4 iv = load_I(y);
#pragma unroll
            for (int c = 0; c < CC; ++c) {
                const f32x4 a = ld4(Ma[c] + (int64_t)y * g.lrs + x0);
                const f32x4 b = ld4(Mb[c] + (int64_t)y * g.lrs + x0);
                store_q(c, y, a * iv + b);
            }
        }
        return;
    } else {
        const int s = S ? S : g.s;
        const int s2 = 2 * s;
        const float inv2s = 1.0f / (float)s2;
        // Horizontal taps: u = (x + 0.5)/s - 0.5 = (2x + 1 - s) / (2s).
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
        // h[c][j]: mean_a, mean_b of low-res row k interpolated at column x0+j
        float ha0[CC][4], hb0[CC][4], ha1[CC][4], hb1[CC][4];
        auto hrow = [&](int k, float (&ha)[CC][4], float (&hb)[CC][4]) {
#pragma unroll
            for (int c = 0; c < CC; ++c) {
                const float *ra = Ma[c] + (int64_t)k * g.lrs;
                const float *rb = Mb[c] + (int64_t)k * g.lrs;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float a0 = ra[xa[j]], a1 = ra[xb[j]];
                    const float b0 = rb[xa[j]], b1 = rb[xb[j]];
                    ha[c][j] = a0 + wx[j] * (a1 - a0);
                    hb[c][j] = b0 + wx[j] * (b1 - b0);
                }
            }
        };
        int k0c = -1, k1c = -1;
        for (int y = yb; y < ye; ++y) {
            const f32x4 iv = load_I(y);
            const int num = 2 * y + 1 - s;
            const int l = floordiv(num, s2);
            const float wy = (float)(num - s2 * l) * inv2s;
            const int k0 = clampi(l, 0, g.Hl - 1), k1 = clampi(l + 1, 0, g.Hl - 1);
            if (k0 != k0c || k1 != k1c) {  // uniform across the wave
                if (k0 == k1c) {
#pragma unroll
                    for (int c = 0; c < CC; ++c)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            ha0[c][j] = ha1[c][j];
                            hb0[c][j] = hb1[c][j];
                        }
                } else {
                    hrow(k0, ha0, hb0);
                }
                if (k1 == k0) {
#pragma unroll
                    for (int c = 0; c < CC; ++c)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            ha1[c][j] = ha0[c][j];
                            hb1[c][j] = hb0[c][j];
                        }
                } else {
                    hrow(k1, ha1, hb1);
                }
                k0c = k0;
                k1c = k1;
            }
#pragma unroll
            for (int c = 0; c < CC; ++c) {
                f32x4 out;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float a = ha0[c][j] + wy * (ha1[c][j] - ha0[c][j]);
                    const float b = hb0[c][j] + wy * (hb1[c][j] - hb0[c][j]);
                    out[j] = a * iv[j] + b;
                }
                store_q(c, y, out);
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

template <typename T>
hipError_t coeff_t(const View &I, const View &P, float *coef, const Geo &g, const TileCfg &t,
                   hipStream_t st) {
    const int ntx = (g.Wl + kTileW - 1) / kTileW;
    const int nty = (g.Hl + t.coeff_th - 1) / t.coeff_th;
    const int ntiles = ntx * nty;
    const size_t lds = coeff_lds_bytes(t.coeff_th, t.coeff_stage, g.R);
    const T *Ip = (const T *)I.data, *Pp = (const T *)P.data;
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_COEFF(TH, STG)                                                                     \
    allow_lds(k_coeff<T, TH, STG>, lds);                                                      \
    hipLaunchKernelGGL((k_coeff<T, TH, STG>), grid, block, lds, st, Ip, I.rs, Pp, P.rs, P.ps, \
                       coef, g, ntx, ntiles)
    if (t.coeff_th == 32) {
        if (t.coeff_stage) { GF_COEFF(32, true); } else { GF_COEFF(32, false); }
    } else {
        if (t.coeff_stage) { GF_COEFF(16, true); } else { GF_COEFF(16, false); }
    }
#undef GF_COEFF
    return hipGetLastError();
}

template <typename T, int CC>
hipError_t output_cc(const View &I, const View &Q, const float *mean, const Geo &g, int c0,
                     const TileCfg &t, bool vec, hipStream_t st) {
    const int ntx = (g.W + kOutTileW - 1) / kOutTileW;
    const int nty = (g.H + 4 * t.out_rows - 1) / (4 * t.out_rows);
    const int ntiles = ntx * nty;
    const T *Ip = (const T *)I.data;
    T *Qp = (T *)Q.data + (int64_t)c0 * Q.ps;
    const dim3 grid(grid8(ntiles)), block(kThreads);
#define GF_OUT(SS)                                                                         \
    hipLaunchKernelGGL((k_output<T, CC, SS>), grid, block, 0, st, Ip, I.rs, Qp, Q.rs, Q.ps, \
                       mean, g, c0, ntx, ntiles, t.out_rows, (int)vec)
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
    const int ntx = (g.Wl + kTileW - 1) / kTileW;
    const int nty = (g.Hl + t.box_th - 1) / t.box_th;
    const int ntiles = ntx * nty;
    const size_t lds = box_lds_bytes(t.box_th, t.box_stage, g.R);
    const dim3 grid(grid8(ntiles), 2 * g.C), block(kThreads);
#define GF_BOX(TH, STG)                 \
    allow_lds(k_box<TH, STG>, lds); \
    hipLaunchKernelGGL((k_box<TH, STG>), grid, block, lds, st, src, dst, g, ntx, ntiles)
    if (t.box_th == 32) {
        if (t.box_stage) { GF_BOX(32, true); } else { GF_BOX(32, false); }
    } else {
        if (t.box_stage) { GF_BOX(16, true); } else { GF_BOX(16, false); }
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
