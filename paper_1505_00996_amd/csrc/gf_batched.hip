// Batched launches: Algorithm 2 for many images of different sizes, channel
// counts, radii and ratios.  Two schedules share one workspace layout and
// one descriptor table:
//
//   phases : one ordinary grid per phase (coefficients, box means, output)
//            over the concatenated tiles of every image -- a fixed handful of
//            launches per batch whatever its size (the output phase is one
//            grid per ratio class); each kernel runs at its own occupancy.
//   queue  : ONE persistent kernel over a queue of tiles, described below.
//
// Queue schedule.
// The queue is phase-major: every coefficient tile of every image (steps
// 1-4), then every box-mean tile (step 5), then every output block (steps
// 6-7).  A workgroup takes the next task with an atomic add on the queue
// head; a task of phase k of image i first waits until all phase k-1 tiles of
// image i are done.  Those tiles sit earlier in the queue, so they were taken
// by workgroups that are running; the earliest unfinished task never waits on
// an unfinished one, so the queue always drains.  The wait is also bounded:
// after a spin limit the workgroup flags an error, skips the task and goes
// on, so every wave reaches the end of the kernel.
//
// Hand-over between workgroups (possibly on different XCDs, whose L2s are
// not coherent with each other): every store of a coefficient or box-mean
// plane and every load of one is a device-coherent access (ldp / stp with
// COH), so no cache-wide writeback or invalidate is needed.  A producer's
// threads wait until their stores have completed, the workgroup meets at a
// barrier and one thread bumps the image's phase counter; a consumer polls
// the counter and only then issues its loads, which are served from the
// coherence point.  (An agent-scope fence per task would write back and
// invalidate the whole L2 of the XCD each time, which costs several times
// the work of a tile.)
#include <hip/hip_runtime.h>

#include "gf_batched.h"
#include "gf_device.h"

namespace gf {
namespace {

using namespace dev;

// Device pointers read from the descriptor table are generic pointers as far
// as the compiler knows, and accesses through generic pointers compile to
// FLAT instructions, which also count against the LDS/scalar wait counter
// and so serialise with every LDS and scalar access.  The images and planes
// are global memory: rebuilding the pointer from its address as a global
// pointer lets the compiler use global loads and stores (a plain cast to the
// global address space and back is folded away).
template <typename T>
__device__ __forceinline__ T *glb(T *p) {
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(uintptr_t)p;
}

// Largest d with D[d].base[ph] <= t (images are laid out in queue order).
__device__ __forceinline__ int find_image(const BDesc *__restrict__ D, int n, int ph, unsigned t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const unsigned b = ph == 0 ? D[mid].base[0] : ph == 1 ? D[mid].base[1] : D[mid].base[2];
        if (b <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The border class is per image, so a task picks its tile code at run time
// (uniform across the workgroup).
template <typename T, int TH, bool COH, int BD>
__device__ __forceinline__ void run_coeff_b(const BDesc &d, int ty0, int tx0, void *lds) {
    const T *I = glb((const T *)d.I), *P = glb((const T *)d.P);
    float *coef = glb(d.coef);
    switch (d.kind) {
        case kSubId:
            coeff_tile<T, kSubId, TH, true, COH, kSubId, BD>(I, d.Irs, P, d.Prs, d.Pps, coef, d.g, ty0, tx0, lds);
            break;
        case kSubNear:
            coeff_tile<T, kSubNear, TH, true, COH, kSubNear, BD>(I, d.Irs, P, d.Prs, d.Pps, coef, d.g, ty0, tx0,
                                                                 lds);
            break;
        default:
            coeff_tile<T, kSubLin, TH, true, COH, kSubLin, BD>(I, d.Irs, P, d.Prs, d.Pps, coef, d.g, ty0, tx0, lds);
            break;
    }
}

template <typename T, int TH, bool COH>
__device__ __forceinline__ void run_coeff(const BDesc &d, unsigned local, void *lds) {
    const int ty0 = ((int)local / d.ntx_l) * TH, tx0 = ((int)local % d.ntx_l) * kTileW;
    if (d.g.border == GF_BORDER_CLIP) run_coeff_b<T, TH, COH, kClip>(d, ty0, tx0, lds);
    else run_coeff_b<T, TH, COH, kPadded>(d, ty0, tx0, lds);
}

template <int TH, bool COH>
__device__ __forceinline__ void run_box(const BDesc &d, unsigned local, void *lds) {
    const unsigned per = (unsigned)(d.ntx_l * d.nty_b);
    const int m = (int)(local / per), r = (int)(local % per);
    const float *src = glb(d.coef) + (int64_t)m * d.g.lps;
    float *dst = glb(d.mean) + (int64_t)m * d.g.lps;
    const int ty0 = (r / d.ntx_l) * TH, tx0 = (r % d.ntx_l) * kTileW;
    if (d.g.border == GF_BORDER_CLIP) box_tile<TH, COH, kClip>(src, dst, d.g, ty0, tx0, lds);
    else box_tile<TH, COH, kPadded>(src, dst, d.g, ty0, tx0, lds);
}

// One output block (32 rows x 256 columns, up to three channels).  The
// workgroup first copies the low-res patch of mean_a and mean_b under the
// block into LDS with coherent loads (each value once), then every lane
// interpolates its 8 x 4 pixels from LDS.  The arithmetic is that of
// output_rows, term for term, so the bits equal those of the per-image
// kernel.  At s = 1 the maps are full resolution and are read directly.
template <typename T>
__device__ __forceinline__ void run_output(const BDesc &d, unsigned local, float *lds) {
    const Geo &g = d.g;
    const unsigned per = (unsigned)(d.ntx_o * d.nty_o);
    const int grp = (int)(local / per), r = (int)(local % per);
    const int c0 = 3 * grp, cc = min(3, g.C - c0);
    const int y0 = (r / d.ntx_o) * (4 * kOutRows), xw = (r % d.ntx_o) * kOutTileW;
    const int lane = threadIdx.x & 63;
    const int yb = y0 + wave_id() * kOutRows, x0 = xw + lane * kOutPx;
    const int nrows = max(0, min(kOutRows, g.H - yb));
    const bool act = x0 < g.W && nrows > 0;
    const bool full = x0 + 3 < g.W;  // one wide access per row, else element-wise
    const T *I = glb((const T *)d.I);
    T *Q = glb((T *)d.Q) + (int64_t)c0 * d.Qps;

    typedef typename Raw4<T>::type raw4;
    raw4 iv[kOutRows];
#pragma unroll
    for (int i = 0; i < kOutRows; ++i) {
        iv[i] = raw4{0, 0, 0, 0};
        if (act && i < nrows) {
            const T *row = I + (int64_t)(yb + i) * d.Irs + x0;
            if (full) {
                iv[i] = ldraw4(row);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (x0 + j < g.W) iv[i][j] = raw1(row + j);
            }
        }
    }
    auto store_q = [&](T *plane, int y, f32x4 v) {
        T *row = plane + (int64_t)y * d.Qrs + x0;
        if (full) {
            st4(row, v);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < g.W) st1(row + j, v[j]);
        }
    };

    const int s = g.s;
    if (s == 1) {  // uniform over the workgroup: no barriers on this path
        if (!act) return;
        for (int c = 0; c < cc; ++c) {
            const float *Ma = glb(d.mean) + (int64_t)(c0 + c) * g.lps;
            const float *Mb = glb(d.mean) + (int64_t)(g.C + c0 + c) * g.lps;
            T *Qc = Q + (int64_t)c * d.Qps;
#pragma unroll
            for (int i = 0; i < kOutRows; ++i) {
                if (i < nrows) {
                    const int64_t o = (int64_t)(yb + i) * g.lrs + x0;
                    f32x4 out;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int jj = x0 + j < g.W ? j : 0;  // stays inside the row
                        out[j] = madd(ldp<true>(Ma + o + jj), widen(iv[i], j), ldp<true>(Mb + o + jj));
                    }
                    store_q(Qc, yb + i, out);
                }
            }
        }
        return;
    }

    const int s2 = 2 * s;
    const float inv2s = 1.0f / (float)s2;
    const int yl = min(y0 + 4 * kOutRows - 1, g.H - 1), xl = min(xw + kOutTileW - 1, g.W - 1);
    const int py0 = clampi(floordiv(2 * y0 + 1 - s, s2), 0, g.Hl - 1);
    const int py1 = clampi(floordiv(2 * yl + 1 - s, s2) + 1, 0, g.Hl - 1);
    const int px0 = clampi(floordiv(2 * xw + 1 - s, s2), 0, g.Wl - 1);
    const int px1 = clampi(floordiv(2 * xl + 1 - s, s2) + 1, 0, g.Wl - 1);
    const int nr = py1 - py0 + 1, nc = px1 - px0 + 1;  // <= kPatchRows, kPatchCols for s >= 2
    float *pa = lds, *pb = lds + kPatchRows * kPatchStride;
    int xa[4], xb[4];
    float wx[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int num = 2 * min(x0 + j, xl) + 1 - s;
        const int l = floordiv(num, s2);
        wx[j] = (float)(num - s2 * l) * inv2s;
        xa[j] = clampi(l, 0, g.Wl - 1) - px0;
        xb[j] = clampi(l + 1, 0, g.Wl - 1) - px0;
    }
    for (int c = 0; c < cc; ++c) {
        const float *Ma = glb(d.mean) + (int64_t)(c0 + c) * g.lps + (int64_t)py0 * g.lrs + px0;
        const float *Mb = glb(d.mean) + (int64_t)(g.C + c0 + c) * g.lps + (int64_t)py0 * g.lrs + px0;
        lds_sync();  // the previous channel's patch has been read
        for (int k = threadIdx.x; k < nr * nc; k += kThreads) {
            const int ry = k / nc, rx = k - ry * nc;
            pa[ry * kPatchStride + rx] = ldp<true>(Ma + (int64_t)ry * g.lrs + rx);
            pb[ry * kPatchStride + rx] = ldp<true>(Mb + (int64_t)ry * g.lrs + rx);
        }
        lds_sync();
        if (act) {
            T *Qc = Q + (int64_t)c * d.Qps;
#pragma unroll
            for (int i = 0; i < kOutRows; ++i) {
                if (i < nrows) {
                    const int num = 2 * (yb + i) + 1 - s;
                    const int l = floordiv(num, s2);
                    const float wy = (float)(num - s2 * l) * inv2s;
                    const int r0 = (clampi(l, 0, g.Hl - 1) - py0) * kPatchStride;
                    const int r1 = (clampi(l + 1, 0, g.Hl - 1) - py0) * kPatchStride;
                    f32x4 out;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float a0 = lerp(pa[r0 + xa[j]], pa[r0 + xb[j]], wx[j]);
                        const float a1 = lerp(pa[r1 + xa[j]], pa[r1 + xb[j]], wx[j]);
                        const float b0 = lerp(pb[r0 + xa[j]], pb[r0 + xb[j]], wx[j]);
                        const float b1 = lerp(pb[r1 + xa[j]], pb[r1 + xb[j]], wx[j]);
                        out[j] = madd(lerp(a0, a1, wy), widen(iv[i], j), lerp(b0, b1, wy));
                    }
                    store_q(Qc, yb + i, out);
                }
            }
        }
    }
}

template <typename T, int TH>
__global__ __launch_bounds__(kThreads) void k_batched(const BDesc *__restrict__ D, int n, unsigned *ctl,
                                                      unsigned total, unsigned p1, unsigned p2,
                                                      unsigned spin_limit) {
    extern __shared__ double lds_d[];
    __shared__ unsigned s_task;
    __shared__ int s_skip;
    unsigned next = 0;  // thread 0: the ticket taken one task ahead
    if (threadIdx.x == 0) s_task = atomicAdd(&ctl[0], 1u);
    __syncthreads();
    for (;;) {
        const unsigned t = s_task;
        if (t >= total) break;  // uniform: every thread read the same s_task
        // Take the next ticket now, so that its round trip overlaps this task.
        // The task it names waits for nothing this one does not, and only
        // ever on tasks before it in the queue, so holding it cannot stall.
        if (threadIdx.x == 0) next = atomicAdd(&ctl[0], 1u);
        const int ph = t < p1 ? 0 : (t < p2 ? 1 : 2);
        const int i = find_image(D, n, ph, t);
        const BDesc &d = D[i];
        const unsigned local = t - (ph == 0 ? d.base[0] : ph == 1 ? d.base[1] : d.base[2]);
        int skip = 0;
        if (ph > 0) {
            // wait until every tile of the previous phase of this image is done
            const unsigned need = ph == 1 ? d.ntiles[0] : d.ntiles[1];
            if (threadIdx.x == 0) {
                unsigned spins = 0;
                int sk = 0;
                while (__hip_atomic_load(&ctl[2 + 2 * i + ph - 1], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > spin_limit) {
                        atomicOr(&ctl[1], 1u);
                        sk = 1;
                        break;
                    }
                }
                s_skip = sk;
            }
            __syncthreads();
            skip = s_skip;
        }
        if (!skip) {
            if (ph == 0) run_coeff<T, TH, true>(d, local, lds_d);
            else if (ph == 1) run_box<TH, true>(d, local, lds_d);
            else run_output<T>(d, local, (float *)lds_d);
            if (ph < 2) {
                // this thread's coherent plane stores have completed ...
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_s_waitcnt(0);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __syncthreads();  // ... and so have every other thread's
                if (threadIdx.x == 0) atomicAdd(&ctl[2 + 2 * i + ph], 1u);
            }
        }
        __syncthreads();  // every thread has read s_task and s_skip
        if (threadIdx.x == 0) s_task = next;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- phases
//
// Task numbering is the queue's: phase k's tasks are [start, start + count)
// with start = 0, p1, p2.  Block -> task goes through xcd_tile, so each XCD
// takes a contiguous run of tasks (whole images, mostly) and their halos
// share its L2.  The kernel boundary orders the phases: plain loads/stores.

// Output block of one image with the per-image kernel's code path (S: the
// compile-time ratio, 0 = read at run time; PX pixels per lane).
template <typename T, int CC, int S, int PX>
__device__ __forceinline__ void out_cc(const BDesc &d, int c0, int yb, int xw) {
    output_rows<T, CC, S, false, PX>(glb((const T *)d.I), d.Irs, glb((T *)d.Q) + (int64_t)c0 * d.Qps, d.Qrs, d.Qps,
                                     glb(d.mean), d.g, c0, yb, xw);
}

template <typename T, int TH>
__global__ __launch_bounds__(kThreads) void k_pcoeff(const BDesc *__restrict__ D, int n, unsigned count) {
    extern __shared__ double lds_d[];
    const unsigned t = (unsigned)xcd_tile((int)blockIdx.x);
    if (t >= count) return;  // uniform per workgroup
    const int i = find_image(D, n, 0, t);
    run_coeff<T, TH, false>(D[i], t - D[i].base[0], lds_d);
}

template <int TH>
__global__ __launch_bounds__(kThreads) void k_pbox(const BDesc *__restrict__ D, int n, unsigned start,
                                                   unsigned count) {
    extern __shared__ double lds_d[];
    const unsigned t = (unsigned)xcd_tile((int)blockIdx.x);
    if (t >= count) return;
    const int i = find_image(D, n, 1, start + t);
    run_box<TH, false>(D[i], start + t - D[i].base[1], lds_d);
}

// fp16 at s = 2 is held to 168 VGPRs (three waves per SIMD instead of two, a
// few values spilled): the 256-image batch 1.937 -> 1.913 ms, the same bits.
// (bf16 at s = 2 would spill over a hundred values; the other ratios already
// fit three.)
template <typename T, int S>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(std::is_same<T, _Float16>::value && S == 2 ? 3 : 1)))
void k_pout(const BDesc *__restrict__ D, int n, unsigned start, unsigned count) {
    constexpr int PX = sizeof(T) == 2 ? 8 : kOutPx;  // out_px(GF_BATCH_PHASES, dtype)
    const unsigned t = (unsigned)xcd_tile((int)blockIdx.x);
    if (t >= count) return;
    const int i = find_image(D, n, 2, start + t);
    const BDesc &d = D[i];
    const unsigned local = start + t - d.base[2];
    const unsigned per = (unsigned)(d.ntx_o * d.nty_o);
    const int grp = (int)(local / per), r = (int)(local % per);
    const int c0 = 3 * grp, cc = min(3, d.g.C - c0);
    const int yb = (r / d.ntx_o) * (4 * kOutRows) + wave_id() * kOutRows, xw = (r % d.ntx_o) * (64 * PX);
    if (cc == 3) out_cc<T, 3, S, PX>(d, c0, yb, xw);
    else if (cc == 2) out_cc<T, 2, S, PX>(d, c0, yb, xw);
    else out_cc<T, 1, S, PX>(d, c0, yb, xw);
}

unsigned grid8u(unsigned n) { return (n + 7u) / 8u * 8u; }

template <typename Kn>
hipError_t allow(Kn k, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// thb: box-mean tile height, TH or 48
template <typename T, int TH>
hipError_t phases_t(int thb, const BDesc *D, int n, unsigned p1, unsigned p2, const OutRanges &out,
                    size_t lds_coeff, size_t lds_box, bool set_lds, hipStream_t st) {
    if (thb != TH && thb != 48) return hipErrorInvalidValue;
    if (set_lds) {
        (void)allow(k_pcoeff<T, TH>, lds_coeff);
        (void)(thb == 48 ? allow(k_pbox<48>, lds_box) : allow(k_pbox<TH>, lds_box));
    }
    const dim3 block(kThreads);
    if (p1) hipLaunchKernelGGL((k_pcoeff<T, TH>), dim3(grid8u(p1)), block, lds_coeff, st, D, n, p1);
    if (p2 > p1) {
        if (thb == 48)
            hipLaunchKernelGGL((k_pbox<48>), dim3(grid8u(p2 - p1)), block, lds_box, st, D, n, p1, p2 - p1);
        else
            hipLaunchKernelGGL((k_pbox<TH>), dim3(grid8u(p2 - p1)), block, lds_box, st, D, n, p1, p2 - p1);
    }
    for (int k = 0; k < kRatioClasses; ++k) {
        const unsigned lo = out.lo[k], cnt = out.hi[k] - out.lo[k];
        if (!cnt) continue;
        const dim3 grid(grid8u(cnt));
        switch (k) {
            case 0: hipLaunchKernelGGL((k_pout<T, 1>), grid, block, kOutResidencyLds, st, D, n, lo, cnt); break;
            case 1: hipLaunchKernelGGL((k_pout<T, 2>), grid, block, kOutResidencyLds, st, D, n, lo, cnt); break;
            case 2: hipLaunchKernelGGL((k_pout<T, 4>), grid, block, kOutResidencyLds, st, D, n, lo, cnt); break;
            case 3: hipLaunchKernelGGL((k_pout<T, 8>), grid, block, kOutResidencyLds, st, D, n, lo, cnt); break;
            default: hipLaunchKernelGGL((k_pout<T, 0>), grid, block, kOutResidencyLds, st, D, n, lo, cnt); break;
        }
    }
    return hipGetLastError();
}

template <typename T, int TH>
hipError_t phases_allow_t(int thb, size_t lds_coeff, size_t lds_box) {
    hipError_t e = allow(k_pcoeff<T, TH>, lds_coeff);
    if (e != hipSuccess) return e;
    return thb == 48 ? allow(k_pbox<48>, lds_box) : allow(k_pbox<TH>, lds_box);
}

// Clears the queue head, the error word and the per-image counters (a kernel
// rather than a memset, so a captured graph replays it correctly).
__global__ void k_zero(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <typename T, int TH>
hipError_t allow_t(size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_batched<T, TH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <typename T, int TH>
hipError_t launch_t(const BDesc *D, int n, unsigned *ctl, unsigned total, unsigned p1, unsigned p2,
                    size_t lds, int grid, bool set_lds, unsigned spin_limit, hipStream_t st) {
    if (set_lds) (void)allow_t<T, TH>(lds);
    hipLaunchKernelGGL((k_batched<T, TH>), dim3(grid), dim3(kThreads), lds, st, D, n, ctl, total, p1, p2,
                       spin_limit);
    return hipGetLastError();
}

template <typename T, int TH>
int occupancy_t(size_t lds) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<T, TH>, kThreads, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_batched(gf_dtype dt, int th, const BDesc *D, int n, unsigned *ctl, unsigned total,
                          unsigned p1, unsigned p2, size_t lds, int grid, bool set_lds, unsigned spin_limit,
                          hipStream_t st) {
    const int nctl = batch_ctl_words(n);
    hipLaunchKernelGGL(k_zero, dim3((nctl + 255) / 256), dim3(256), 0, st, ctl, nctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define GF_B(TT)                                                                                       \
    return th == 8 ? launch_t<TT, 8>(D, n, ctl, total, p1, p2, lds, grid, set_lds, spin_limit, st)     \
         : th == 16 ? launch_t<TT, 16>(D, n, ctl, total, p1, p2, lds, grid, set_lds, spin_limit, st)   \
                    : launch_t<TT, 24>(D, n, ctl, total, p1, p2, lds, grid, set_lds, spin_limit, st)
    switch (dt) {
        case GF_F32: GF_B(float);
        case GF_F16: GF_B(_Float16);
        case GF_BF16: GF_B(dev::bf16);
    }
#undef GF_B
    return hipErrorInvalidValue;
}

hipError_t batched_allow_lds(gf_dtype dt, int th, size_t lds) {
#define GF_A(TT) return th == 8 ? allow_t<TT, 8>(lds) : th == 16 ? allow_t<TT, 16>(lds) : allow_t<TT, 24>(lds)
    switch (dt) {
        case GF_F32: GF_A(float);
        case GF_F16: GF_A(_Float16);
        case GF_BF16: GF_A(dev::bf16);
    }
#undef GF_A
    return hipErrorInvalidValue;
}

hipError_t launch_phases(gf_dtype dt, int th, int thb, const BDesc *D, int n, unsigned *ctl, unsigned p1, unsigned p2,
                         const OutRanges &out, size_t lds_coeff, size_t lds_box, bool set_lds, hipStream_t st) {
    // the error word reads 0 after a phase-schedule launch as well
    const int nctl = batch_ctl_words(n);
    hipLaunchKernelGGL(k_zero, dim3((nctl + 255) / 256), dim3(256), 0, st, ctl, nctl);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define GF_P(TT)                                                                                    \
    switch (th) {                                                                                   \
        case 8: return phases_t<TT, 8>(thb, D, n, p1, p2, out, lds_coeff, lds_box, set_lds, st);    \
        case 16: return phases_t<TT, 16>(thb, D, n, p1, p2, out, lds_coeff, lds_box, set_lds, st);  \
        case 24: return phases_t<TT, 24>(thb, D, n, p1, p2, out, lds_coeff, lds_box, set_lds, st);  \
        case 32: return phases_t<TT, 32>(thb, D, n, p1, p2, out, lds_coeff, lds_box, set_lds, st);  \
        case 48: return phases_t<TT, 48>(thb, D, n, p1, p2, out, lds_coeff, lds_box, set_lds, st);  \
    }                                                                                               \
    return hipErrorInvalidValue
    switch (dt) {
        case GF_F32: GF_P(float);
        case GF_F16: GF_P(_Float16);
        case GF_BF16: GF_P(dev::bf16);
    }
#undef GF_P
    return hipErrorInvalidValue;
}

hipError_t phases_allow_lds(gf_dtype dt, int th, int thb, size_t lds_coeff, size_t lds_box) {
#define GF_PA(TT)                                                    \
    switch (th) {                                                    \
        case 8: return phases_allow_t<TT, 8>(thb, lds_coeff, lds_box);    \
        case 16: return phases_allow_t<TT, 16>(thb, lds_coeff, lds_box);  \
        case 24: return phases_allow_t<TT, 24>(thb, lds_coeff, lds_box);  \
        case 32: return phases_allow_t<TT, 32>(thb, lds_coeff, lds_box);  \
        case 48: return phases_allow_t<TT, 48>(thb, lds_coeff, lds_box);  \
    }                                                                \
    return hipErrorInvalidValue
    switch (dt) {
        case GF_F32: GF_PA(float);
        case GF_F16: GF_PA(_Float16);
        case GF_BF16: GF_PA(dev::bf16);
    }
#undef GF_PA
    return hipErrorInvalidValue;
}

int batched_occupancy(gf_dtype dt, int th, size_t lds) {
#define GF_O(TT) \
    return th == 8 ? occupancy_t<TT, 8>(lds) : th == 16 ? occupancy_t<TT, 16>(lds) : occupancy_t<TT, 24>(lds)
    switch (dt) {
        case GF_F32: GF_O(float);
        case GF_F16: GF_O(_Float16);
        case GF_BF16: GF_O(dev::bf16);
    }
#undef GF_O
    return 1;
}

}  // namespace gf
