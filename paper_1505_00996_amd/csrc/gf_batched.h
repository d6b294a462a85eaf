// Shared host/device layout of the persistent batched launch.  Not public ABI.
#pragma once

#include <stdint.h>

#include "gf_internal.h"

namespace gf {

// One image of a batch, as the persistent kernel reads it (device memory).
struct BDesc {
    const void *I, *P;
    void *Q;
    float *coef, *mean;  // 2C planes each, in the workspace
    int64_t Irs, Prs, Pps, Qrs, Qps;
    Geo g;
    int kind;                // subsampling kind (0 identity, 1 nearest, 2 two-tap mean)
    int ntx_l, nty_l;        // low-res tiles: 64 columns x TH rows
    int nty_b;               // rows of box-mean tiles (64 columns x the plan's box tile height)
    int ntx_o, nty_o;        // output blocks: 64 * out_px(schedule, dtype) columns x 32 rows
    unsigned base[3];        // queue index of the image's first task in each phase
    unsigned ntiles[3];      // tasks of each phase: tiles, 2C*tiles, groups*blocks
};

// Pixels per lane of the output blocks: the phase schedule's output grids
// take 16-bit rows eight pixels at a time (one 16-byte access per row, as
// the per-image kernel does); the queue kernel's output tasks stage a
// 256-column patch and take four.
inline int out_px(int schedule, gf_dtype dt) { return schedule == GF_BATCH_PHASES && dt != GF_F32 ? 8 : kOutPx; }

// The control words live at the start of the batch workspace: [0] queue
// head, [1] error flag, then 2 per image: coefficient tiles done, box tiles
// done.
inline int batch_ctl_words(int n) { return 2 + 2 * n; }

// Images of a plan are ordered by ratio class (s = 1, 2, 4, 8, any other),
// so each class's output blocks are one contiguous range of the queue and
// the phase schedule runs them with the per-image kernel's compile-time
// taps: class k covers queue indices [lo[k], hi[k]).
constexpr int kRatioClasses = 5;
inline int ratio_class(int s) { return s == 1 ? 0 : s == 2 ? 1 : s == 4 ? 2 : s == 8 ? 3 : 4; }
struct OutRanges {
    unsigned lo[kRatioClasses], hi[kRatioClasses];
};

// Low-res patch under one output block (32 x 256 pixels) at s >= 2: rows
// span at most ceil(31/s) + 2 <= 18 and columns ceil(255/s) + 2 <= 130.
constexpr int kPatchRows = 18, kPatchCols = 130, kPatchStride = kPatchCols + 1;
constexpr size_t kOutPatchLds = 2 * kPatchRows * kPatchStride * sizeof(float);

// Clears the control words, then launches the persistent kernel.  With
// set_lds the kernel's dynamic-LDS limit is raised first (otherwise
// batched_allow_lds must have been called for this dtype, th and size).
// spin_limit: polls of each bounded wait before the tile gives up.
hipError_t launch_batched(gf_dtype dt, int th, const BDesc *D, int n, unsigned *ctl, unsigned total,
                          unsigned p1, unsigned p2, size_t lds, int grid, bool set_lds, unsigned spin_limit,
                          hipStream_t st);
hipError_t batched_allow_lds(gf_dtype dt, int th, size_t lds);

// Phase schedule: clears the control words, then the three phase grids on
// st (coefficient tiles [0, p1),
// box tiles [p1, p2), output blocks [p2, total)).  With set_lds the kernels'
// dynamic-LDS limits are raised first (else phases_allow_lds must have run).
hipError_t launch_phases(gf_dtype dt, int th, int thb, const BDesc *D, int n, unsigned *ctl, unsigned p1, unsigned p2,
                         const OutRanges &out, size_t lds_coeff, size_t lds_box, bool set_lds, hipStream_t st);
hipError_t phases_allow_lds(gf_dtype dt, int th, int thb, size_t lds_coeff, size_t lds_box);
int batched_occupancy(gf_dtype dt, int th, size_t lds);

}  // namespace gf
