// Persistent batched launch: Algorithm 2 for many images of different sizes,
// channel counts, radii and ratios in ONE kernel over a queue of tiles.
//
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
// Memory ordering between workgroups (possibly on different XCDs, whose L2s
// are not coherent with each other): a producer's threads fence at agent
// scope after their stores (release: stores reach memory, L2 written back),
// then one thread bumps the image's phase counter; the consumer polls the
// counter and fences at agent scope (acquire: stale L1/L2 lines dropped)
// before reading.
#include <hip/hip_runtime.h>

#include "gf_batched.h"
#include "gf_device.h"

namespace gf {
namespace {

using namespace dev;

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

template <typename T, int TH>
__device__ __forceinline__ void run_coeff(const BDesc &d, unsigned local, void *lds) {
    const unsigned per = (unsigned)(d.ntx_l * d.nty_l);
    const int c = (int)(local / per), r = (int)(local % per);
    const int ty0 = (r / d.ntx_l) * TH, tx0 = (r % d.ntx_l) * kTileW;
    const T *I = (const T *)d.I;
    const T *Pc = (const T *)d.P + (int64_t)c * d.Pps;
    float *ac = d.coef + (int64_t)c * d.g.lps, *bc = d.coef + (int64_t)(d.g.C + c) * d.g.lps;
    switch (d.kind) {
        case kSubId: coeff_tile<T, kSubId, TH, true>(I, d.Irs, Pc, d.Prs, ac, bc, d.g, ty0, tx0, lds); break;
        case kSubNear: coeff_tile<T, kSubNear, TH, true>(I, d.Irs, Pc, d.Prs, ac, bc, d.g, ty0, tx0, lds); break;
        default: coeff_tile<T, kSubLin, TH, true>(I, d.Irs, Pc, d.Prs, ac, bc, d.g, ty0, tx0, lds); break;
    }
}

template <int TH>
__device__ __forceinline__ void run_box(const BDesc &d, unsigned local, void *lds) {
    const unsigned per = (unsigned)(d.ntx_l * d.nty_l);
    const int m = (int)(local / per), r = (int)(local % per);
    box_tile<TH>(d.coef + (int64_t)m * d.g.lps, d.mean + (int64_t)m * d.g.lps, d.g, (r / d.ntx_l) * TH,
                 (r % d.ntx_l) * kTileW, lds);
}

// Output blocks use the run-time-ratio form of output_rows: one code path
// for every s keeps the persistent kernel's register budget (and so its
// occupancy during the HBM-bound phase) at that of a single variant.
template <typename T>
__device__ __forceinline__ void run_output(const BDesc &d, unsigned local) {
    const unsigned per = (unsigned)(d.ntx_o * d.nty_o);
    const int grp = (int)(local / per), r = (int)(local % per);
    const int c0 = 3 * grp, cc = min(3, d.g.C - c0);
    const int yb = (r / d.ntx_o) * (4 * kOutRows) + wave_id() * kOutRows, xw = (r % d.ntx_o) * kOutTileW;
    const T *I = (const T *)d.I;
    T *Q = (T *)d.Q + (int64_t)c0 * d.Qps;
    const bool vec = d.vec != 0;
    if (cc == 3) output_rows<T, 3, 0>(I, d.Irs, Q, d.Qrs, d.Qps, d.mean, d.g, c0, yb, xw, vec);
    else if (cc == 2) output_rows<T, 2, 0>(I, d.Irs, Q, d.Qrs, d.Qps, d.mean, d.g, c0, yb, xw, vec);
    else output_rows<T, 1, 0>(I, d.Irs, Q, d.Qrs, d.Qps, d.mean, d.g, c0, yb, xw, vec);
}

template <typename T, int TH>
__global__ __launch_bounds__(kThreads) void k_batched(const BDesc *__restrict__ D, int n, unsigned *ctl,
                                                      unsigned total, unsigned p1, unsigned p2,
                                                      unsigned spin_limit) {
    extern __shared__ double lds_d[];
    __shared__ unsigned s_task;
    __shared__ int s_skip;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(&ctl[0], 1u);
        __syncthreads();
        const unsigned t = s_task;
        if (t >= total) break;  // uniform: every thread read the same s_task
        const int ph = t < p1 ? 0 : (t < p2 ? 1 : 2);
        const int i = find_image(D, n, ph, t);
        const BDesc &d = D[i];
        const unsigned local = t - (ph == 0 ? d.base[0] : ph == 1 ? d.base[1] : d.base[2]);
        if (ph > 0) {
            // wait until every tile of the previous phase of this image is done
            const unsigned need = ph == 1 ? d.ntiles[0] : d.ntiles[1];
            if (threadIdx.x == 0) {
                unsigned spins = 0;
                int skip = 0;
                while (__hip_atomic_load(&ctl[2 + 2 * i + ph - 1], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > spin_limit) {
                        atomicOr(&ctl[1], 1u);
                        skip = 1;
                        break;
                    }
                }
                s_skip = skip;
            }
            __syncthreads();
            __threadfence();  // acquire: drop stale cached lines before reading the previous phase
            if (s_skip) {
                __syncthreads();
                continue;
            }
        }
        if (ph == 0) run_coeff<T, TH>(d, local, lds_d);
        else if (ph == 1) run_box<TH>(d, local, lds_d);
        else run_output<T>(d, local);
        if (ph < 2) {
            __threadfence();  // release: this thread's stores reach memory before the count
            __syncthreads();
            if (threadIdx.x == 0) atomicAdd(&ctl[2 + 2 * i + ph], 1u);
        }
        __syncthreads();  // s_task / s_skip are rewritten by the next iteration
    }
}

// Clears the queue head, the error word and the per-image counters (a kernel
// rather than a memset, so a captured graph replays it correctly).
__global__ void k_zero(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <typename T, int TH>
hipError_t launch_t(const BDesc *D, int n, unsigned *ctl, unsigned total, unsigned p1, unsigned p2,
                    size_t lds, int grid, hipStream_t st) {
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_batched<T, TH>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_batched<T, TH>), dim3(grid), dim3(kThreads), lds, st, D, n, ctl, total, p1, p2,
                       kBatchSpinLimit);
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
                          unsigned p1, unsigned p2, size_t lds, int grid, hipStream_t st) {
    const int nctl = batch_ctl_words(n);
    hipLaunchKernelGGL(k_zero, dim3((nctl + 255) / 256), dim3(256), 0, st, ctl, nctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define GF_B(TT)                                                                           \
    return th == 8 ? launch_t<TT, 8>(D, n, ctl, total, p1, p2, lds, grid, st)              \
         : th == 16 ? launch_t<TT, 16>(D, n, ctl, total, p1, p2, lds, grid, st)            \
                    : launch_t<TT, 24>(D, n, ctl, total, p1, p2, lds, grid, st)
    switch (dt) {
        case GF_F32: GF_B(float);
        case GF_F16: GF_B(_Float16);
        case GF_BF16: GF_B(dev::bf16);
    }
#undef GF_B
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
