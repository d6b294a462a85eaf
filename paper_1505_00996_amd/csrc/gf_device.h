// Device code of the (fast) guided filter for gfx950 (CDNA4, wave64): the
// per-tile work of Algorithm 2 of He & Sun, "Fast Guided Filter", written as
// device functions so that the per-image kernels (gf_kernels.hip) and the
// persistent batched kernel (gf_batched.hip) run the same code.
//
//   coeff_tile  : subsample I and p (step 1) while staging a low-res tile and
//                 its r' halo in LDS; window sums of I', I'^2, p', I'p'
//                 (step 2); var, cov (step 3) and a, b of Eqs. 2-3 (step 4).
//   box_tile    : box mean of one coefficient map (step 5), clip-normalised
//                 or over the map padded by replication / reflect-101.
//   output_rows : bilinear upsampling of mean_a, mean_b fused with
//                 q = mean_a * I + mean_b against the full-resolution I
//                 (steps 6-7); the HBM-bound pass.
//
// Every tile function is called by a whole 256-thread workgroup (4 waves);
// coeff_tile and box_tile use workgroup barriers (lds_sync) and LDS passed in by the caller.
//
// Window sums: a row pass (each thread slides a (2r'+1)-wide window over
// kRun consecutive outputs of one region row) writes row sums to LDS; a
// column pass (each thread owns one column and TH/4 consecutive output rows)
// slides over them.  The statistics of step 2 are summed in FP64: in a flat
// window mean(I*I) - mean(I)^2 and mean(I*p) - mean(I) mean(p) cancel almost
// completely, FP64 leaves ~1e-16 of rounding there (FP32 would leave ~1e-8,
// which moves a by percent at eps = 1e-6), and products of FP32 samples are
// exact in FP64.  On gfx950 an FP64 add or FMA issues at the rate of a
// non-packed FP32 one.  Samples are also shifted by the tile's first sample,
// which keeps the sums small.  The box means of a and b have no cancellation
// and are summed in FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "gf_internal.h"

namespace gf {
namespace dev {

// Floating-point expressions in this file (and in the kernels that include
// it) are evaluated as written: no multiply and add are fused unless an fma
// is spelled out.  The same tile code is inlined into several kernels, and
// left to itself the compiler fuses differently in each, so one pixel could
// get different bits from the per-image and the batched launches.
#pragma clang fp contract(off)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// The same vectors at element alignment, for accesses to rows of I, p and q,
// whose starts are only element-aligned.  HSA runs gfx950 with unaligned
// global accesses enabled, so such an access is still one wide instruction
// at any element-aligned address (at about 80% of the aligned rate when it
// straddles a 4-byte boundary, against a quarter or less for element-wise
// accesses).
typedef float f32x4e __attribute__((ext_vector_type(4), aligned(4)));
typedef _Float16 f16x4e __attribute__((ext_vector_type(4), aligned(2)));
typedef unsigned short u16x4e __attribute__((ext_vector_type(4), aligned(2)));
typedef float f32x2e __attribute__((ext_vector_type(2), aligned(4)));
typedef _Float16 f16x2e __attribute__((ext_vector_type(2), aligned(2)));
typedef unsigned short u16x2e __attribute__((ext_vector_type(2), aligned(2)));

struct bf16 {
    unsigned short bits;
};

// ---------------------------------------------------------------- storage

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float((unsigned)v.bits << 16); }

// float -> bfloat16, round to nearest even (gfx950 converts in hardware).
__device__ __forceinline__ unsigned short f32_to_bf16_bits(float f) {
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
// q is an FP32 result rounded once more, to nearest even, for 16-bit
// storage.  The empty asm pins the FP32 value: without it the compiler may
// fuse the last multiply-add with the narrowing (v_fma_mixlo_f16, one
// rounding straight to fp16), and whether it does differs between kernels,
// so the same pixel could get different bits in different launches.
__device__ __forceinline__ float pin_f32(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)pin_f32(v); }
template <> __device__ __forceinline__ bf16 from_f32<bf16>(float v) { return bf16{f32_to_bf16_bits(v)}; }

template <typename T> __device__ __forceinline__ float ld(const T *p) { return to_f32(*p); }

// Four consecutive elements, 16 bytes (fp32) or 8 bytes (16-bit), in one
// access at any element-aligned address.
__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4e *)p; }
__device__ __forceinline__ f32x4 ld4(const _Float16 *p) {
    f16x4 h = *(const f16x4e *)p;
    return f32x4{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
}
__device__ __forceinline__ f32x4 ld4(const bf16 *p) {
    u16x4 b = *(const u16x4e *)p;
    return f32x4{__uint_as_float((unsigned)b.x << 16), __uint_as_float((unsigned)b.y << 16),
                 __uint_as_float((unsigned)b.z << 16), __uint_as_float((unsigned)b.w << 16)};
}

// Streaming (non-temporal) stores of four outputs, one access at any
// element-aligned address.
__device__ __forceinline__ void st4(float *p, f32x4 v) {
    __builtin_nontemporal_store((f32x4e)v, (f32x4e *)p);
}
__device__ __forceinline__ void st4(_Float16 *p, f32x4 v) {
    f16x4e h = {from_f32<_Float16>(v.x), from_f32<_Float16>(v.y), from_f32<_Float16>(v.z),
                from_f32<_Float16>(v.w)};
    __builtin_nontemporal_store(h, (f16x4e *)p);
}
__device__ __forceinline__ void st4(bf16 *p, f32x4 v) {
    u16x4e b = {f32_to_bf16_bits(v.x), f32_to_bf16_bits(v.y), f32_to_bf16_bits(v.z),
                f32_to_bf16_bits(v.w)};
    __builtin_nontemporal_store(b, (u16x4e *)p);
}
template <typename T> __device__ __forceinline__ void st1(T *p, float v) { *p = from_f32<T>(v); }

// Two consecutive elements in one access at any element-aligned address.
__device__ __forceinline__ f32x2 ld2(const float *p) { return *(const f32x2e *)p; }
__device__ __forceinline__ f32x2 ld2(const _Float16 *p) {
    f16x2 h = *(const f16x2e *)p;
    return f32x2{(float)h.x, (float)h.y};
}
__device__ __forceinline__ f32x2 ld2(const bf16 *p) {
    u16x2 b = *(const u16x2e *)p;
    return f32x2{__uint_as_float((unsigned)b.x << 16), __uint_as_float((unsigned)b.y << 16)};
}

// Four samples held in their storage width (half the registers for 16-bit
// types) and widened when used; widening is exact.
template <typename T> struct Raw4;
template <> struct Raw4<float> { typedef f32x4 type; };
template <> struct Raw4<_Float16> { typedef f16x4 type; };
template <> struct Raw4<bf16> { typedef u16x4 type; };
__device__ __forceinline__ f32x4 ldraw4(const float *p) { return *(const f32x4e *)p; }
__device__ __forceinline__ f16x4 ldraw4(const _Float16 *p) { return *(const f16x4e *)p; }
__device__ __forceinline__ u16x4 ldraw4(const bf16 *p) { return *(const u16x4e *)p; }
__device__ __forceinline__ float raw1(const float *p) { return *p; }
__device__ __forceinline__ _Float16 raw1(const _Float16 *p) { return *p; }
__device__ __forceinline__ unsigned short raw1(const bf16 *p) { return p->bits; }
__device__ __forceinline__ float widen(f32x4 v, int j) { return v[j]; }
__device__ __forceinline__ float widen(f16x4 v, int j) { return (float)v[j]; }
__device__ __forceinline__ float widen(u16x4 v, int j) { return __uint_as_float((unsigned)v[j] << 16); }

// Accesses to the low-resolution planes that workgroups of one launch hand
// to each other (the batched kernel).  With COH they are relaxed atomics at
// agent scope, which the compiler emits as device-coherent loads and stores
// (sc1): a store is written through the XCD's L2 and is complete when its
// vmcnt retires, and a load is served from the coherence point, not from a
// line another XCD's write has made stale.  Handing planes over this way
// needs no cache-wide writeback or invalidate (an agent-scope fence does
// both), only a wait for the producer's stores before it signals.
typedef __attribute__((address_space(1))) float gfloat;  // global memory, not generic
template <bool COH> __device__ __forceinline__ float ldp(const float *p) {
    if constexpr (COH)
        return __hip_atomic_load((gfloat *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH> __device__ __forceinline__ void stp(float *p, float v) {
    if constexpr (COH) __hip_atomic_store((gfloat *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

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

// Border classes of the window-sum tiles, fixed per kernel so the clip
// path carries no code of the others:
//   kClip   the window's in-map samples only (outside ones weigh 0), mean
//           over their count;
//   kPadded the map extended past its edges as g.border says (replicate or
//           reflect-101), mean over (2r'+1)^2.
constexpr int kClip = 0, kPadded = 1;

// Index that position i of an n-long map axis reads under a padded border.
// Replicate clamps.  Reflect-101 applies the reflection about both ends,
// F(m) = (n-1) - |(n-1) - |m||, which is exact for -(n-1) <= m <= 2(n-1),
// `reps` times (reps > 1 only for windows wider than the axis; the host
// counts them), then clamps, which also makes a one-pixel axis read its
// pixel and keeps the rows a ragged tile reads past its outputs in bounds.
__device__ __forceinline__ int pad_index(int i, int n, int border, int reps) {
    if (border == GF_BORDER_REFLECT101) {
        int m = n - 1 - abs(n - 1 - abs(i));
        for (int t = 1; t < reps; ++t) m = n - 1 - abs(n - 1 - abs(m));
        i = m;
    }
    return clampi(i, 0, n - 1);
}
template <int BD>
__device__ __forceinline__ int window_len(int i, int R, int n) {
    return BD == kClip ? clip_len(i, R, n) : 2 * R + 1;
}

// Wave index as a scalar, so values derived from it stay in SGPRs.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

// Approximate reciprocal (1 ulp): the results it feeds tolerate 1e-7.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Workgroup barrier that orders LDS accesses only.  A thread's outstanding
// global loads stay in flight across it; __syncthreads also waits for them
// (its fence covers all memory), which would cancel the prefetches the tile
// code issues ahead of LDS passes.  Every barrier in the tile code only
// separates LDS writers from LDS readers.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// a + w (b - a) and a x + b, each with one fused rounding
__device__ __forceinline__ float lerp(float a, float b, float w) { return __builtin_fmaf(w, b - a, a); }
__device__ __forceinline__ float madd(float a, float x, float b) { return __builtin_fmaf(a, x, b); }

// ---------------------------------------------------------------- sampling
//
// Algorithm 2 step 1, the low-res sample at (ly, lx) inside [0,Hl) x [0,Wl).
// The kind is fixed per launch, so the loads carry no data-dependent branch:
//   kSubId   s = 1: the image itself;
//   kSubNear nearest: full-res s*ly + floor(s/2), clamped to the image (also
//            bilinear with odd s, whose sample centre falls on a pixel);
//   kSubLin  bilinear with even s: the mean of the two pixels on each side
//            of the low-res centre s*ly + (s-1)/2, taps clamped.
// A sample is split into a row part (uniform across a wave in the fills, so
// the row address stays scalar) and a column part (per lane).
constexpr int kSubId = 0, kSubNear = 1, kSubLin = 2;

struct Taps {
    int a, b;  // full-res indices (b only used by kSubLin)
};

template <int K>
__device__ __forceinline__ Taps taps(int l, int s, int n) {
    if constexpr (K == kSubId) {
        return Taps{l, l};
    } else if constexpr (K == kSubNear) {
        return Taps{min(s * l + (s >> 1), n - 1), 0};
    } else {
        return Taps{min(s * l + (s >> 1) - 1, n - 1), min(s * l + (s >> 1), n - 1)};
    }
}

template <int K, typename T>
__device__ __forceinline__ float sample_rc(const T *__restrict__ img, int64_t rs, Taps ry, Taps cx) {
    const T *r0 = img + (int64_t)ry.a * rs;
    if constexpr (K != kSubLin) {
        return ld(r0 + cx.a);
    } else {
        const T *r1 = img + (int64_t)ry.b * rs;
        const float v00 = ld(r0 + cx.a), v01 = ld(r0 + cx.b);
        const float v10 = ld(r1 + cx.a), v11 = ld(r1 + cx.b);
        return 0.5f * (0.5f * v00 + 0.5f * v01) + 0.5f * (0.5f * v10 + 0.5f * v11);
    }
}

template <int K, typename T>
__device__ __forceinline__ float sample(const T *__restrict__ img, int64_t rs, int ly, int lx,
                                        const Geo &g) {
    return sample_rc<K>(img, rs, taps<K>(ly, g.s, g.H), taps<K>(lx, g.s, g.W));
}

// ---------------------------------------------------------------- window sums

constexpr int kFillRows = 8;   // region rows per wave per fill batch

// Stage an SH x SW region whose element (ry, rx) is f(ry, rx, c_ry, c_rx):
// wave w takes rows w, w+4, ...; lanes take columns lane and lane + 64 (and
// further chunks for wide regions); kFillRows rows x 2 chunks of loads are
// issued before the first LDS store.  Out-of-range rows/columns are clamped
// so every load is unconditional; f decides the value kept.
template <class F>
__device__ __forceinline__ void fill_tile(float *dst, int SH, int SW, int SWp, F f) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    for (int c0 = 0; c0 < SW; c0 += 128) {
        const int rx0 = c0 + lane, rx1 = c0 + 64 + lane;
        for (int r0 = wave; r0 < SH; r0 += 4 * kFillRows) {
            float v0[kFillRows], v1[kFillRows];
#pragma unroll
            for (int b = 0; b < kFillRows; ++b) {
                const int ry = min(r0 + 4 * b, SH - 1);
                v0[b] = f(ry, min(rx0, SW - 1));
                v1[b] = f(ry, min(rx1, SW - 1));
            }
#pragma unroll
            for (int b = 0; b < kFillRows; ++b) {
                const int ry = r0 + 4 * b;
                if (ry < SH) {
                    if (rx0 < SW) dst[ry * SWp + rx0] = v0[b];
                    if (rx1 < SW) dst[ry * SWp + rx1] = v1[b];
                }
            }
        }
    }
}

// A region of at most 4*kFillRows rows and 128 columns is one fill batch; its
// loads can be issued early into registers (fill_load) and written to LDS
// later (fill_store), so their latency overlaps other work.  Same data and
// placement as fill_tile.
struct FillRegs {
    float v0[kFillRows], v1[kFillRows];
};
__host__ __device__ constexpr bool one_fill_batch(int SH, int SW) { return SH <= 4 * kFillRows && SW <= 128; }
template <class F>
__device__ __forceinline__ void fill_load(FillRegs &r, int SH, int SW, F f) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int cx0 = min(lane, SW - 1), cx1 = min(64 + lane, SW - 1);
#pragma unroll
    for (int b = 0; b < kFillRows; ++b) {
        const int ry = min(wave + 4 * b, SH - 1);
        r.v0[b] = f(ry, cx0);
        r.v1[b] = f(ry, cx1);
    }
}
__device__ __forceinline__ void fill_store(const FillRegs &r, float *dst, int SH, int SW, int SWp) {
    const int lane = threadIdx.x & 63, wave = wave_id();
#pragma unroll
    for (int b = 0; b < kFillRows; ++b) {
        const int ry = wave + 4 * b;
        if (ry < SH) {
            if (lane < SW) dst[ry * SWp + lane] = r.v0[b];
            if (64 + lane < SW) dst[ry * SWp + 64 + lane] = r.v1[b];
        }
    }
}

// Two regions of the same shape in one batch (twice the loads in flight).
template <class F1, class F2>
__device__ __forceinline__ void fill_tile2(float *d1, float *d2, int SH, int SW, int SWp, F1 f1, F2 f2) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    for (int c0 = 0; c0 < SW; c0 += 128) {
        const int rx0 = c0 + lane, rx1 = c0 + 64 + lane;
        const int cx0 = min(rx0, SW - 1), cx1 = min(rx1, SW - 1);
        for (int r0 = wave; r0 < SH; r0 += 4 * kFillRows) {
            float a0[kFillRows], a1[kFillRows], b0[kFillRows], b1[kFillRows];
#pragma unroll
            for (int b = 0; b < kFillRows; ++b) {
                const int ry = min(r0 + 4 * b, SH - 1);
                a0[b] = f1(ry, cx0);
                a1[b] = f1(ry, cx1);
                b0[b] = f2(ry, cx0);
                b1[b] = f2(ry, cx1);
            }
#pragma unroll
            for (int b = 0; b < kFillRows; ++b) {
                const int ry = r0 + 4 * b;
                if (ry < SH) {
                    if (rx0 < SW) {
                        d1[ry * SWp + rx0] = a0[b];
                        d2[ry * SWp + rx0] = b0[b];
                    }
                    if (rx1 < SW) {
                        d1[ry * SWp + rx1] = a1[b];
                        d2[ry * SWp + rx1] = b1[b];
                    }
                }
            }
        }
    }
}

// n^2 var and n^2 cov are the two cancelling differences; they are taken
// in FP64, everything after them in FP32.  Eqs. 2-3.
__device__ __forceinline__ void coeff_from_sums(int n, double Su, double Suu, double Sv, double Suv,
                                                float cI, float cP, float eps, float &a, float &b) {
    const double nd = (double)n;
    const float n2var = (float)fmax(nd * Suu - Su * Su, 0.0);
    const float n2cov = (float)(nd * Suv - Su * Sv);
    const float rn = rcp((float)n);
    const float var = n2var * rn * rn;
    const float cov = n2cov * rn * rn;  // Eq. 2 numerator
    const float mI = cI + (float)Su * rn, mp = cP + (float)Sv * rn;
    a = cov * rcp(var + eps);  // Eq. 2
    b = mp - a * mI;           // Eq. 3
}

// One TH x 64 tile of a_c, b_c (low-res) at tile origin (ty0, tx0) for every
// channel c of p (planes P + c*Pps; a_c at coef + c*lps, b_c at
// coef + (C+c)*lps).  The guide's window statistics (sums of u and u*u) are
// formed once and kept in registers; then, channel by channel, those of p
// (sums of v and u*v) and the coefficients.  LDS holds two FP64 row-sum
// planes at a time.  With STAGE the samples of the region are staged in LDS
// first (the guide's once, each channel's in turn); without it (large r',
// where the staged region would not fit) the row pass reads them through the
// caches.
// KP: how p is sampled -- like I (Algorithm 2), or kSubId when p is given at
// low resolution already (joint upsampling: its rows are the low-res rows).
// BD: border class (kClip, kPadded).
// [cb, ce): the channels of p this tile serves (ce < 0: through C - 1).
template <typename T, int K, int TH, bool STAGE, bool COH = false, int KP = K, int BD = kClip>
__device__ __forceinline__ void coeff_tile(const T *__restrict__ I, int64_t Irs,
                                           const T *__restrict__ P, int64_t Prs, int64_t Pps,
                                           float *__restrict__ coef, const Geo &g, int ty0, int tx0,
                                           void *lds, int cb = 0, int ce = -1) {
    constexpr int LC = TH / 4;  // output rows per thread in the column pass
    const int R = g.R, SH = TH + 2 * R, SW = kTileW + 2 * R, SWp = region_stride(R);
    const int plane = SH * kRowW;
    double *rA = (double *)lds, *rB = rA + plane;
    float *sU = (float *)(rB + plane), *sV = sU + SH * SWp;
    const int oy = ty0 - R, ox = tx0 - R;
    const int lane = threadIdx.x & 63, wave = wave_id();

    // u = I' - cI and v = p' - cP over the region; outside the low-res map
    // 0 (kClip) or the sample the border extension puts there (kPadded).
    // The clip case multiplies by 0 rather than selecting: a select on a
    // loaded value lets the compiler turn the load into a branch that waits
    // for it, one load at a time.  The sample read there is an in-image one
    // (clamped address), so the product is an exact 0 for finite images.
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
    const float cI = sample<K>(I, Irs, ty0, tx0, g);
    auto gU = [&](int ry, int rx) { return gsample(KI{}, I, Irs, cI, ry, rx); };

    const int col = lane, r0 = wave * LC;
    const int lx = tx0 + col;
    const int nx = window_len<BD>(lx, R, g.Wl);

    // (Window loops have a run-time length 2r'+1; unrolling them keeps several
    // LDS reads in flight instead of one read-wait-add per element.  The
    // additions stay in the same order.)
    // Row pass: rA = sum x, rB = sum u*x over each run of kRun outputs, with
    // x = u (PAIR false) or x = v (PAIR true, v from gV / sV).
    auto row_pass = [&](auto pair, auto gV) {
        constexpr bool PAIR = decltype(pair)::value;
        for (int it = threadIdx.x; it < SH * (kTileW / kRun); it += kThreads) {
            // consecutive lanes take consecutive rows of the same run: region
            // reads stride SWp (odd) and row-sum writes 2*kRowW words, which
            // spread over the LDS banks (lanes on one row would collide)
            const int j0 = (it / SH) * kRun, ry = it - (it / SH) * SH;
            const float *pu = sU + ry * SWp + j0, *pv = sV + ry * SWp + j0;
            auto U = [&](int k) -> float { return STAGE ? pu[k] : gU(ry, j0 + k); };
            auto V = [&](int k) -> float { return STAGE ? pv[k] : gV(ry, j0 + k); };
            // every read of the run before any write (see box_tile)
            float uin[kRun], uout[kRun], xin[kRun], xout[kRun];
#pragma unroll
            for (int t = 1; t < kRun; ++t) {
                uin[t] = U(t + 2 * R);
                uout[t] = U(t - 1);
                xin[t] = PAIR ? V(t + 2 * R) : uin[t];
                xout[t] = PAIR ? V(t - 1) : uout[t];
            }
            double A = 0.0, B = 0.0;
#pragma unroll 8
            for (int k = 0; k <= 2 * R; ++k) {
                const double u = U(k);
                const double x = PAIR ? (double)V(k) : u;
                A += x;
                B = __builtin_fma(u, x, B);
            }
            double ra[kRun], rb[kRun];
            ra[0] = A;
            rb[0] = B;
#pragma unroll
            for (int t = 1; t < kRun; ++t) {
                const double ui = uin[t], uo = uout[t], xi = xin[t], xo = xout[t];
                A += xi - xo;
                B += __builtin_fma(ui, xi, -uo * xo);
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

    const int cend = ce < 0 ? g.C : ce;
    const T *P0 = P + (int64_t)cb * Pps;
    const float cP0 = sample<KP>(P0, Prs, ty0, tx0, g);
    auto gV0 = [&](int ry, int rx) { return gsample(KQ{}, P0, Prs, cP0, ry, rx); };
    if (STAGE) {
        fill_tile2(sU, sV, SH, SW, SWp, gU, gV0);  // guide and channel 0 in one batch
        lds_sync();
    }

    // guide: sums of u and u*u, once for all channels
    double Su[LC], Suu[LC];
    row_pass(std::false_type{}, gV0);
    lds_sync();
    {
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
            Su[t] = A;
            Suu[t] = B;
        }
    }

    // When a region is one fill batch, the next channel's samples are loaded
    // while this channel's passes run.
    const bool ahead = STAGE && one_fill_batch(SH, SW);
    FillRegs next;
    float cPn = 0.f;
    for (int c = cb; c < cend; ++c) {
        const T *Pc = P + (int64_t)c * Pps;
        const float cP = c != cb ? cPn : cP0;
        auto gV = [&](int ry, int rx) { return gsample(KQ{}, Pc, Prs, cP, ry, rx); };
        // sV is free: the last row pass that read it ended at a barrier
        if (STAGE && c != cb) {
            if (ahead) fill_store(next, sV, SH, SW, SWp);
            else fill_tile(sV, SH, SW, SWp, gV);
        }
        lds_sync();  // sV staged; the previous column pass is done with rA, rB
        if (c + 1 < cend) {
            const T *Pn = Pc + Pps;
            cPn = sample<KP>(Pn, Prs, ty0, tx0, g);
            if (ahead) fill_load(next, SH, SW, [&](int ry, int rx) { return gsample(KQ{}, Pn, Prs, cPn, ry, rx); });
        }
        // sums of v and u*v, then a and b
        row_pass(std::true_type{}, gV);
        lds_sync();
        float *ac = coef + (int64_t)c * g.lps, *bc = coef + (int64_t)(g.C + c) * g.lps;
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
            const int ly = ty0 + r0 + t;
            if (ly < g.Hl && lx < g.Wl) {
                float a, b;
                coeff_from_sums(window_len<BD>(ly, R, g.Hl) * nx, Su[t], Suu[t], A, B, cI, cP, g.eps, a, b);
                stp<COH>(ac + (int64_t)ly * g.lrs + lx, a);
                stp<COH>(bc + (int64_t)ly * g.lrs + lx, b);
            }
        }
    }
}

// One TH x 64 tile of the box mean of a low-res FP32 plane (border class BD).
template <int TH, bool COH = false, int BD = kClip>
__device__ __forceinline__ void box_tile(const float *__restrict__ S, float *__restrict__ D,
                                         const Geo &g, int ty0, int tx0, void *lds) {
    constexpr int LC = TH / 4;
    const int R = g.R, SH = TH + 2 * R, SW = kTileW + 2 * R, SWp = region_stride(R);
    float *rA = (float *)lds;
    float *sX = rA + SH * kRowW;
    const int oy = ty0 - R, ox = tx0 - R;
    const int lane = threadIdx.x & 63, wave = wave_id();
    fill_tile(sX, SH, SW, SWp, [&](int ry, int rx) -> float {
        const int ly = oy + ry, lx = ox + rx;
        if constexpr (BD == kClip) {
            const bool in = ly >= 0 && ly < g.Hl && lx >= 0 && lx < g.Wl;
            const float v = ldp<COH>(S + (int64_t)clampi(ly, 0, g.Hl - 1) * g.lrs + clampi(lx, 0, g.Wl - 1));
            return v * (in ? 1.f : 0.f);  // product, not select: see coeff_tile
        } else {
            return ldp<COH>(S + (int64_t)pad_index(ly, g.Hl, g.border, g.refl_h) * g.lrs +
                            pad_index(lx, g.Wl, g.border, g.refl_w));
        }
    });
    lds_sync();
    for (int it = threadIdx.x; it < SH * (kTileW / kRun); it += kThreads) {
        const int j0 = (it / SH) * kRun, ry = it - (it / SH) * SH;  // lanes down the rows (see coeff_tile)
        const float *px = sX + ry * SWp + j0;
        // every read of the run before any write: the row sums share LDS
        // with the region, so a write between reads would order them
        float xin[kRun], xout[kRun], res[kRun];
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            xin[t] = px[t + 2 * R];
            xout[t] = px[t - 1];
        }
        float A = 0.f;
#pragma unroll 8
        for (int k = 0; k <= 2 * R; ++k) A += px[k];
        res[0] = A;
#pragma unroll
        for (int t = 1; t < kRun; ++t) {
            A += xin[t] - xout[t];
            res[t] = A;
        }
        float *oa = rA + ry * kRowW + j0;
#pragma unroll
        for (int t = 0; t < kRun; ++t) oa[t] = res[t];
    }
    lds_sync();
    const int col = lane, r0 = wave * LC;
    const int lx = tx0 + col;
    const int nx = window_len<BD>(lx, R, g.Wl);
    float A = 0.f;
#pragma unroll 8
    for (int k = 0; k <= 2 * R; ++k) A += rA[(r0 + k) * kRowW + col];
#pragma unroll
    for (int t = 0; t < LC; ++t) {
        if (t) A += rA[(r0 + t + 2 * R) * kRowW + col] - rA[(r0 + t - 1) * kRowW + col];
        const int ly = ty0 + r0 + t;
        if (ly < g.Hl && lx < g.Wl)
            stp<COH>(D + (int64_t)ly * g.lrs + lx, A * rcp((float)(window_len<BD>(ly, R, g.Hl) * nx)));
    }
}

// ---------------------------------------------------------------- output
//
// A wave covers kOutRows = 8 rows starting at a multiple of 8 and 64 PX
// full-res columns, PX pixels per lane: 4 for fp32 and 8 for 16-bit storage
// in the per-image kernel and the batched output grids, so that every row
// access is 16 bytes (the queue kernel's output blocks use 4).  A lane first
// loads its 8 x PX guide pixels (all loads in flight together); then,
// channel by channel, it loads the low-res rows and columns of mean_a,
// mean_b its pixels interpolate from, interpolates them horizontally once,
// and for every row finishes the bilinear weights and writes q = a*I + b
// with non-temporal stores.
//
// Upsampling geometry (half-pixel centres): full-res x maps to low-res
// u = (x + 0.5)/s - 0.5 = (2x + 1 - s) / (2s), taps floor(u), floor(u) + 1
// clamped to the map.  For s in {2, 4, 8} lanes start at x0 = 0 mod PX and
// waves at y = 0 mod 8, so which low-res rows/columns each pixel uses,
// relative to the first one, is known at compile time.

constexpr int kOutRows = 8;

// floor((2x + 1 - s) / (2s)) and its fractional part, for compile-time use
constexpr int cfloor_u(int x, int s) {
    return (2 * x + 1 - s) >= 0 ? (2 * x + 1 - s) / (2 * s) : -((2 * s - 1 - (2 * x + 1 - s)) / (2 * s));
}
constexpr float cfrac_u(int x, int s) {
    return (float)((2 * x + 1 - s) - 2 * s * cfloor_u(x, s)) / (float)(2 * s);
}

// Rows of PX pixels per lane.  fp32 (PX = 4): FP32 values, one 16-byte
// access.  16-bit (PX = 8): the 8 stored values kept in their storage width
// (half the registers) and widened, exactly, when used; one 16-byte access.
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8e __attribute__((ext_vector_type(8), aligned(2)));
template <typename T, int PX>
struct PixRow {
    float v[PX];
    __device__ __forceinline__ float at(int j) const { return v[j]; }
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int j = 0; j < PX; ++j) v[j] = 0.f;
    }
};
template <typename T>
struct PixRow<T, 8> {
    static_assert(sizeof(T) == 2, "8-wide rows are 16-bit rows");
    u16x8 b;
    __device__ __forceinline__ float at(int j) const {
        if constexpr (std::is_same<T, bf16>::value) return __uint_as_float((unsigned)b[j] << 16);
        else return (float)__builtin_bit_cast(_Float16, (unsigned short)b[j]);
    }
    __device__ __forceinline__ void zero() { b = u16x8{0, 0, 0, 0, 0, 0, 0, 0}; }
};
__device__ __forceinline__ unsigned short raw16(const _Float16 *p) {
    return __builtin_bit_cast(unsigned short, *p);
}
__device__ __forceinline__ unsigned short raw16(const bf16 *p) { return p->bits; }
// one row of PX consecutive elements at `row`: one wide access (full: all
// PX lie in the image), or one element at a time up to n (0 past it)
template <typename T, int PX>
__device__ __forceinline__ void ld_row(PixRow<T, PX> &r, const T *row, bool full, int n) {
    if constexpr (PX == 4) {
        if (full) {
            const f32x4 a = ld4(row);
#pragma unroll
            for (int j = 0; j < 4; ++j) r.v[j] = a[j];
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) r.v[j] = j < n ? ld(row + j) : 0.f;
        }
    } else {
        if (full) {
            r.b = *(const u16x8e *)row;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) r.b[j] = j < n ? raw16(row + j) : (unsigned short)0;
        }
    }
}
template <int PX, typename T>
__device__ __forceinline__ void stv(T *p, const float *v) {
    if constexpr (PX == 4) {
        st4(p, f32x4{v[0], v[1], v[2], v[3]});
    } else {
        static_assert(PX == 8 && sizeof(T) == 2, "8-wide rows are 16-bit rows");
        u16x8 b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (std::is_same<T, bf16>::value) b[j] = f32_to_bf16_bits(v[j]);
            else b[j] = __builtin_bit_cast(unsigned short, from_f32<_Float16>(v[j]));
        }
        __builtin_nontemporal_store((u16x8e)b, (u16x8e *)p);
    }
}

// The NC low-res values of one map row a lane interpolates from (columns
// cx[0..NC-1]): for NC >= 4 and `contig` (no tap clamped, cx consecutive)
// in 16- and 8-byte loads at any element-aligned address, else one at a
// time.  The values are the same either way.  (Four or more taps per row
// come with s = 2, and with s = 4 at 8 pixels per lane: there the vector
// loads cut the batched s = 2 output grid from 375 to 291 us; with three
// taps, 8-byte loads at odd element offsets were slower than three
// 4-byte ones: 40.2 against 37.3 us on the 4000x3000 fp32 output pass.)
template <int NC>
__device__ __forceinline__ void ld_taps(const float *row, const int (&cx)[NC], bool contig, float (&v)[NC]) {
    if (NC >= 4 && contig) {
        const float *p = row + cx[0];
        int k = 0;
#pragma unroll
        for (; k + 4 <= NC; k += 4) {
            const f32x4 a = *(const f32x4e *)(p + k);
            v[k] = a[0];
            v[k + 1] = a[1];
            v[k + 2] = a[2];
            v[k + 3] = a[3];
        }
#pragma unroll
        for (; k + 2 <= NC; k += 2) {
            const f32x2 a = *(const f32x2e *)(p + k);
            v[k] = a[0];
            v[k + 1] = a[1];
        }
        if (k < NC) v[k] = p[k];
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = row[cx[k]];
    }
}

// q for CC channels (planes Q + c*Qps) of the wave's 8 x (64 PX) block at
// (yb, xw), PX pixels per lane; mean_a_c = M + (c0+c)*lps,
// mean_b_c = M + (C+c0+c)*lps.  S: compile-time ratio, 0 = read g.s at run
// time.  Every pixel gets the same arithmetic whatever PX is.
// EPI (detail enhancement): with P the c0-th plane of p (same layout as Q),
// each output becomes e = q + gain (p - q), formed from the FP32 q before
// the store's rounding.
template <typename T, int CC, int S, bool EPI = false, int PX = kOutPx>
__device__ __forceinline__ void output_rows(const T *__restrict__ I, int64_t Irs, T *__restrict__ Q,
                                            int64_t Qrs, int64_t Qps, const float *__restrict__ M,
                                            const Geo &g, int c0, int yb, int xw,
                                            const T *__restrict__ P = nullptr, int64_t Prs = 0,
                                            int64_t Pps = 0, float gain = 0.f) {
    static_assert(PX == 4 || PX == 8, "4 or 8 pixels per lane");
    constexpr int ROWS = kOutRows;
    const int lane = threadIdx.x & 63;
    const int x0 = xw + lane * PX;
    const int nrows = min(ROWS, g.H - yb);
    if (x0 >= g.W || nrows <= 0) return;  // no barriers below
    // Per row: one wide access per lane (whatever the row start's
    // alignment), or one element at a time for the lane at the row's end.
    const bool full = x0 + PX - 1 < g.W;

    typedef PixRow<T, PX> Row;
    auto load_row = [&](const T *plane, int64_t rs, int y, Row &r) {
        ld_row<T, PX>(r, plane + (int64_t)y * rs + x0, full, g.W - x0);
    };
    Row iv[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        if (i < nrows) load_row(I, Irs, yb + i, iv[i]);
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
    // the rows of channel c of p, for the detail epilogue (loaded together)
    Row pv[EPI ? ROWS : 1];
    pv[0].zero();
    auto load_p = [&](int c) {
        if constexpr (EPI) {
            const T *Pc = P + (int64_t)c * Pps;
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) load_row(Pc, Prs, yb + i, pv[i]);
                else pv[i].zero();
            }
        }
    };
    auto finish = [&](float *q, const Row &pr) {
        if constexpr (EPI) {
#pragma unroll
            for (int j = 0; j < PX; ++j) q[j] = lerp(q[j], pr.at(j), gain);
        }
    };

    if constexpr (S == 1) {
        // Algorithm 1: the maps are full resolution; rows are padded to a
        // multiple of 16 floats, so the 16-byte reads at x0 stay in the row.
#pragma unroll 1
        for (int c = 0; c < CC; ++c) {
            const float *Ma = M + (int64_t)(c0 + c) * g.lps;
            const float *Mb = M + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * Qps;
            load_p(c);
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                if (i < nrows) {
                    const int y = yb + i;
                    float out[PX];
#pragma unroll
                    for (int j = 0; j < PX; j += 4) {
                        const f32x4 a = ld4(Ma + (int64_t)y * g.lrs + x0 + j);
                        const f32x4 b = ld4(Mb + (int64_t)y * g.lrs + x0 + j);
#pragma unroll
                        for (int k = 0; k < 4; ++k) out[j + k] = madd(a[k], iv[i].at(j + k), b[k]);
                    }
                    finish(out, pv[EPI ? i : 0]);
                    store_q(Qc, y, out);
                }
            }
        }
    } else if constexpr (S == 2 || S == 4 || S == 8) {
        // low-res rows base_y .. base_y + NL - 1 and columns base_x .. base_x + NC - 1
        constexpr int NL = cfloor_u(ROWS - 1, S) - cfloor_u(0, S) + 2;
        constexpr int NC = cfloor_u(PX - 1, S) - cfloor_u(0, S) + 2;
        const int base_y = floordiv(2 * yb + 1 - S, 2 * S);
        const int base_x = floordiv(2 * x0 + 1 - S, 2 * S);
        int ry[NL], cx[NC];
#pragma unroll
        for (int m = 0; m < NL; ++m) ry[m] = clampi(base_y + m, 0, g.Hl - 1);
#pragma unroll
        for (int m = 0; m < NC; ++m) cx[m] = clampi(base_x + m, 0, g.Wl - 1);
        // no tap clamped: the NC values of a row are consecutive (vector loads)
        const bool contig = cx[NC - 1] == cx[0] + NC - 1;
        // horizontal weights and taps: compile time when s divides x0 (PX = 8,
        // or s < 8); at s = 8 with four pixels per lane they depend on whether
        // the lane starts at 0 or 4 mod 8, and the taps do not (offset 0)
        constexpr bool XPHASE = S == 8 && PX == 4;
        float wx[PX];
#pragma unroll
        for (int j = 0; j < PX; ++j)
            wx[j] = XPHASE ? (float)((2 * ((x0 & 7) + j) + 1 - 8) & 15) * (1.0f / 16.0f) : cfrac_u(j, S);
#pragma unroll 1
        for (int c = 0; c < CC; ++c) {
            const float *Ma = M + (int64_t)(c0 + c) * g.lps;
            const float *Mb = M + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * Qps;
            load_p(c);
            // the low-res values under the block, all loads in flight together
            float va[NL][NC], vb[NL][NC];
#pragma unroll
            for (int m = 0; m < NL; ++m) {
                ld_taps<NC>(Ma + (int64_t)ry[m] * g.lrs, cx, contig, va[m]);
                ld_taps<NC>(Mb + (int64_t)ry[m] * g.lrs, cx, contig, vb[m]);
            }
            // horizontal interpolation of low-res row m at pixel j
            auto hlerp = [&](const float (&v)[NL][NC], int m, int j) -> float {
                const int k0 = XPHASE ? 0 : cfloor_u(j, S) - cfloor_u(0, S);
                return lerp(v[m][k0], v[m][k0 + 1], wx[j]);
            };
            // four pixels per lane: every row's horizontal values once, then
            // the rows; eight: the two rows each output row needs, per row
            // (same values, fewer live registers)
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
                    finish(out, pv[EPI ? i : 0]);
                    store_q(Qc, yb + i, out);
                }
            }
        }
    } else {
        // any other ratio: taps computed per pixel and per row at run time
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
                float iy[PX];
#pragma unroll
                for (int j = 0; j < PX; ++j) iy[j] = 0.f;
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    if (r == i) {
#pragma unroll
                        for (int j = 0; j < PX; ++j) iy[j] = iv[r].at(j);
                    }
                float out[PX];
#pragma unroll
                for (int j = 0; j < PX; ++j) {
                    const float a0 = lerp(ra0[xa[j]], ra0[xb[j]], wx[j]);
                    const float a1 = lerp(ra1[xa[j]], ra1[xb[j]], wx[j]);
                    const float b0 = lerp(rb0[xa[j]], rb0[xb[j]], wx[j]);
                    const float b1 = lerp(rb1[xa[j]], rb1[xb[j]], wx[j]);
                    out[j] = madd(lerp(a0, a1, wy), iy[j], lerp(b0, b1, wy));
                }
                if constexpr (EPI) {
                    Row pr;
                    load_row(P + (int64_t)c * Pps, Prs, y, pr);
                    finish(out, pr);
                }
                store_q(Qc, y, out);
            }
        }
    }
}

// Workgroups are handed to the 8 XCDs round robin (id mod 8).  Launches use
// a grid that is a multiple of 8 and this map gives XCD k the k-th
// contiguous range of logical tiles (row-major), so tiles that share halo
// rows of the low-res maps share an L2.
__device__ __forceinline__ int xcd_tile(int bid) {
    const int per = (int)gridDim.x >> 3;
    return (bid & 7) * per + (bid >> 3);
}

}  // namespace dev
}  // namespace gf
