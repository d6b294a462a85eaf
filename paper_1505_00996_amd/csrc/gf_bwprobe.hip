// Attainable-bandwidth probes for measurement (libgf_bwprobe.so, used by
// bench.py; not part of the filter library).  They move the same kind of
// traffic as the fused upsample + output pass (Algorithm 2 steps 6-7) with
// the same access shape and nothing else, so their rate is the ceiling that
// pass can be held to on this GPU:
//   gfbw_r1w3 : read one fp32 H x W plane, write three (q_c = k_c I + b_c, one
//               FMA per element), 16-byte accesses, non-temporal stores, the
//               output kernel's workgroup shape (four waves side by side, 8
//               rows x 256 columns each) and XCD-aware block order;
//   gfbw_copy : a plain 16-byte-vector copy of n floats (n a multiple of 4).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4e __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ int xcd_block(int bid) {
    const int per = (int)gridDim.x >> 3;
    return (bid & 7) * per + (bid >> 3);
}

__global__ __launch_bounds__(256) void k_r1w3(const float *__restrict__ I, float *__restrict__ Q, int H, int W,
                                              int64_t ps, int ntx, int nblocks) {
    const int b = xcd_block(blockIdx.x);
    if (b >= nblocks) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int y0 = (b / ntx) * 8, x0 = ((b % ntx) * 4 + wave) * 256 + lane * 4;
    const int nrows = min(8, H - y0);
    if (x0 >= W) return;
    const bool full = x0 + 3 < W;
    f32x4 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        v[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (i < nrows) {
            const float *row = I + (int64_t)(y0 + i) * W + x0;
            if (full) {
                v[i] = *(const f32x4e *)row;
            } else {
                for (int j = 0; j < 4; ++j)
                    if (x0 + j < W) v[i][j] = row[j];
            }
        }
    }
    const float k[3] = {0.5f, 0.75f, 1.25f}, o[3] = {0.125f, 0.25f, -0.5f};
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        float *Qc = Q + (int64_t)c * ps;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < nrows) {
                f32x4 q;
#pragma unroll
                for (int j = 0; j < 4; ++j) q[j] = __builtin_fmaf(k[c], v[i][j], o[c]);
                float *row = Qc + (int64_t)(y0 + i) * W + x0;
                if (full) {
                    __builtin_nontemporal_store((f32x4e)q, (f32x4e *)row);
                } else {
                    for (int j = 0; j < 4; ++j)
                        if (x0 + j < W) row[j] = q[j];
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(src[i], dst + i);
}

}  // namespace

extern "C" {

// Q: three planes of h x w floats, plane stride h*w; device pointers.
int gfbw_r1w3(const float *I, float *Q, int h, int w, void *stream) {
    if (!I || !Q || h < 1 || w < 1) return -1;
    const int ntx = (w + 1023) / 1024, nty = (h + 7) / 8, nblocks = ntx * nty;
    const int grid = (nblocks + 7) / 8 * 8;
    hipLaunchKernelGGL(k_r1w3, dim3(grid), dim3(256), 0, (hipStream_t)stream, I, Q, h, w, (int64_t)h * w, ntx,
                       nblocks);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// n floats, n a multiple of 4; 16-byte aligned device pointers.
int gfbw_copy(const float *src, float *dst, int64_t n, void *stream) {
    if (!src || !dst || n < 4 || n % 4 || ((uintptr_t)src | (uintptr_t)dst) % 16) return -1;
    hipLaunchKernelGGL(k_copy, dim3(256 * 16), dim3(256), 0, (hipStream_t)stream, (const f32x4 *)src, (f32x4 *)dst,
                       n / 4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
