// Host planning of the persistent batched launch (shared by gf_fast_batched
// and the request engine).  Not public ABI.
#pragma once

#include <vector>

#include "gf.h"
#include "gf_batched.h"

namespace gf {

struct BatchPlan {
    int n = 0;
    gf_dtype dtype = GF_F32;
    int sched = GF_BATCH_PHASES;
    int th = 0;               // tile height of the window-sum tiles (0: use per-image launches)
    int thb = 0;              // rows of the box-mean tiles (th, or 48 under the phase schedule)
    size_t lds = 0;           // dynamic LDS of the persistent kernel (queue schedule)
    size_t lds_coeff = 0, lds_box = 0;  // dynamic LDS of the phase kernels
    size_t desc_off = 0;      // byte offset of the descriptor table in the workspace
    size_t ws_bytes = 0;      // workspace bytes the plan needs
    unsigned p1 = 0, p2 = 0, total = 0;  // queue: [0,p1) coefficients, [p1,p2) box means, [p2,total) output
    OutRanges out{};          // output blocks of each ratio class
    std::vector<BDesc> desc;  // in plan order: images sorted by ratio class
    std::vector<int> order;   // order[k] = caller's index of desc[k]
};

// Validate the n problems and lay out the queue and the workspace (whose
// device base address is ws_base; may be null when only sizes are wanted).
gf_status plan_batch(int n, const gf_image *I, const gf_image *p, const gf_image *q,
                     const gf_params *pr, char *ws_base, const gf_batch_cfg &cfg, BatchPlan *plan);

// The context's batch configuration (the default without a context).
gf_batch_cfg ctx_batch_cfg(gf_ctx *ctx);
bool batch_cfg_ok(const gf_batch_cfg &c);

// Tile heights {coefficients, box means} a batch whose largest low-res
// radius is maxR gets ({0, 0}: none fits).
TileCfg batch_tiles(const gf_batch_cfg &cfg, int maxR);

// Upload the descriptor table and enqueue the persistent kernel on st.
gf_status launch_plan(gf_ctx *ctx, BatchPlan &plan, void *ws, hipStream_t st);

}  // namespace gf
