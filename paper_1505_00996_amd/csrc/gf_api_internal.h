// Host-side internals shared by the API translation units (not public ABI).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "gf.h"
#include "gf_internal.h"

namespace gf {
class Engine;
}

struct gf_ctx {
    int device = 0;
    void *ws = nullptr;      // workspace for calls that pass none
    size_t ws_bytes = 0;
    std::mutex tune_mu;      // guards `tuned`
    std::unordered_map<uint64_t, gf::TileCfg> tuned;  // tile shapes picked by gf_tune
    gf::Engine *engine = nullptr;  // request interface (gf_submit / gf_poll)
    gf_batch_cfg batch_cfg{GF_BATCH_PHASES, 0};  // batched launches (gf_ctx_set_batch_cfg / gf_tune_batched)
    std::atomic<uint32_t> spin_limit{gf::kBatchSpinLimit};  // bounded waits of the queue schedule
    std::atomic<int> fuse{GF_FUSE_AUTO};  // box means fused into the output pass (gf_ctx_set_fusion)
    // kernel timing (gf_ctx_profile)
    bool profiling = false;
    struct Mark {
        int kernel;
        hipEvent_t start, end;
    };
    std::mutex prof_mu;
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
    // pinned staging of batched-launch descriptor tables
    std::mutex pin_mu;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t pin_ev = nullptr;  // completes when the last upload from `pin` is done
};

namespace gf {

gf_status fail(gf_status st, const char *fmt, ...);
const char *last_error();
int lowres_radius(int r, int s);
bool tiles_fit(const Geo &g, const TileCfg &t);
size_t workspace_bytes(const Geo &g);
// p_low: p is the low-resolution input of joint upsampling (ceil(h/s) x ceil(w/s)).
gf_status validate(const gf_image *I, const gf_image *p, const gf_image *q, const gf_params *pr,
                   bool p_low = false);
gf_status run_fast(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                   const gf_params *pr, void *ws, size_t ws_bytes, hipStream_t st,
                   const TileCfg *tiles, bool p_low = false, const float *gain = nullptr);

// Timing of one launcher call when the context is profiling (no-op
// otherwise).  By default events are recorded on the stream before and after
// the scope; with `in_dispatch` the scope only hands out a Stamp whose events
// the launcher puts into the kernel dispatches, and the caller reports
// whether the launch went through (commit) so only recorded events are read.
struct ProfScope {
    gf_ctx *ctx;
    int kernel;
    hipStream_t st;
    bool in_dispatch;
    bool committed = false;
    hipEvent_t start = nullptr, end = nullptr;
    ProfScope(gf_ctx *c, int k, hipStream_t s, bool in_dispatch = false);
    ~ProfScope();
    Stamp stamp() const { return Stamp{start, end}; }
    void commit(bool ok) { committed = ok; }
};
gf_status ctx_use_device(gf_ctx *ctx);
gf_status ctx_workspace(gf_ctx *ctx, size_t need, void **ws);
bool ctx_tiles(gf_ctx *ctx, const gf_image *I, const gf_image *p, const gf_params *pr,
               TileCfg *out);
uint64_t tile_key(gf_dtype dt, int h, int w, int C, int r, int s);
TileCfg default_tiles(const Geo &g);
gf_status engine_start(gf_ctx *ctx, size_t arena_bytes, int max_inflight);
// Looks up the current device's fixed scratch array of gf_fast_noalloc.
gf_status noalloc_prepare();
void engine_stop(gf_ctx *ctx);

}  // namespace gf
