// A stand-in for the HIP runtime and the kernel launchers, so that the host
// code of libgf.so (validation, planning, the request engine, autotuners,
// tuning files) can be built with sanitizers and run on a machine without a
// GPU.  "Device" memory is host memory, copies are memcpy, streams run
// nothing, events complete when recorded, and every kernel launch succeeds
// without computing anything.  The batched launchers clear the control words
// as the real ones do, and can be told to set the error word (fake_fail_next),
// which exercises the engine's error path.  Not part of the library.
#include <hip/hip_runtime_api.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <set>

#include "gf_batched.h"
#include "gf_internal.h"

struct ihipStream_t {
    int id;
};
struct ihipEvent_t {
    bool recorded;
};

namespace {
std::mutex g_mu;
std::set<void *> g_dev, g_host;  // live allocations
std::atomic<int> g_launches{0};
}  // namespace

std::atomic<int> fake_fail_next{0};  // batched launches that set their error word

int fake_launches() { return g_launches.load(); }
size_t fake_live_allocations() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_dev.size() + g_host.size();
}

static void *alloc256(size_t n) { return aligned_alloc(256, (n + 255) / 256 * 256 + 256); }

extern "C" {

hipError_t hipMalloc(void **ptr, size_t size) {
    if (!ptr) return hipErrorInvalidValue;
    *ptr = alloc256(size);
    if (!*ptr) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mu);
    g_dev.insert(*ptr);
    return hipSuccess;
}
hipError_t hipFree(void *ptr) {
    if (!ptr) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev.erase(ptr)) return hipErrorInvalidValue;
    free(ptr);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int) {
    if (!ptr) return hipErrorInvalidValue;
    *ptr = alloc256(size);
    if (!*ptr) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mu);
    g_host.insert(*ptr);
    return hipSuccess;
}
hipError_t hipHostFree(void *ptr) {
    if (!ptr) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_host.erase(ptr)) return hipErrorInvalidValue;
    free(ptr);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t) {
    if (n && (!dst || !src)) return hipErrorInvalidValue;
    memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) {
    *s = new ihipStream_t{1};
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) { return hipStreamCreate(s); }
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new ihipEvent_t{false};
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (!e) return hipErrorInvalidValue;
    e->recorded = true;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) { return e && e->recorded ? hipSuccess : hipErrorNotReady; }
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!ms || !a || !b) return hipErrorInvalidValue;
    *ms = 0.001f * (float)(((uintptr_t)a ^ (uintptr_t)b) % 97 + 1);  // distinct, deterministic per pair
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int *n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }

}  // extern "C"

namespace gf {

static hipError_t launched() {
    ++g_launches;
    return hipSuccess;
}

hipError_t launch_coeff(gf_dtype, const View &, const View &, float *, const Geo &, const TileCfg &, hipStream_t,
                        const Stamp &, bool) {
    return launched();
}
hipError_t launch_box(const float *, float *, const Geo &, const TileCfg &, hipStream_t, const Stamp &) {
    return launched();
}
hipError_t launch_area(gf_dtype, const View &, const View &, bool, float *, const Geo &, hipStream_t,
                       const Stamp &) {
    return launched();
}
hipError_t launch_coeff_lowres(const float *, const float *, float *, const Geo &, const TileCfg &, hipStream_t,
                               const Stamp &) {
    return launched();
}
hipError_t launch_output(gf_dtype, const View &, const View &, const float *, const Geo &, const TileCfg &,
                         hipStream_t, const Stamp &, const Detail &) {
    return launched();
}
hipError_t launch_coeff_color(gf_dtype, const View &, const View &, float *, const Geo &, const TileCfg &,
                              hipStream_t, const Stamp &, bool) {
    return launched();
}
hipError_t launch_coeff_color_lowres(const float *, const float *, float *, const Geo &, const TileCfg &,
                                     hipStream_t, const Stamp &) {
    return launched();
}
hipError_t launch_outbox(gf_dtype, const View &, const View &, const float *, const Geo &, const TileCfg &, int,
                         hipStream_t, const Stamp &, const Detail &) {
    return launched();
}
hipError_t launch_output_color(gf_dtype, const View &, const View &, const float *, const Geo &, hipStream_t,
                               const Stamp &, const Detail &) {
    return launched();
}

// The batched launchers clear the control words first, as k_zero does.
static void clear_ctl(unsigned *ctl, int n) {
    memset(ctl, 0, sizeof(unsigned) * batch_ctl_words(n));
    if (fake_fail_next.load() > 0) {
        --fake_fail_next;
        ctl[1] = 1u;  // a tile gave up its wait
    }
}
hipError_t launch_batched(gf_dtype, int, const BDesc *, int n, unsigned *ctl, unsigned, unsigned, unsigned,
                          size_t, int grid, bool, unsigned, hipStream_t) {
    if (grid < 1) return hipErrorInvalidValue;
    clear_ctl(ctl, n);
    return launched();
}
hipError_t batched_allow_lds(gf_dtype, int, size_t lds) { return lds <= kLdsLimit ? hipSuccess : hipErrorInvalidValue; }
hipError_t launch_phases(gf_dtype, int, int, const BDesc *, int n, unsigned *ctl, unsigned, unsigned,
                         const OutRanges &, size_t, size_t, bool, hipStream_t) {
    clear_ctl(ctl, n);
    return launched();
}
hipError_t phases_allow_lds(gf_dtype, int, int, size_t a, size_t b) {
    return a <= kLdsLimit && b <= kLdsLimit ? hipSuccess : hipErrorInvalidValue;
}
int batched_occupancy(gf_dtype, int, size_t) { return 2; }
// The fixed scratch array of gf_fast_noalloc lives in device code, not built here.
gf_status noalloc_prepare() { return GF_OK; }

}  // namespace gf
