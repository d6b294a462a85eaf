// Request interface (gf_submit / gf_poll): continuous batching on one GPU.
//
// gf_submit validates a request, checks that its workspace could ever fit
// the context's device arena (else GF_ENOMEM) and that fewer than
// max_inflight requests are held (else GF_EBUSY), queues it and returns a
// ticket.  A worker thread owned by the context:
//   * retires finished batches (hipEventQuery on each in-flight batch),
//     frees their arena ranges and wakes pollers;
//   * admits queued requests in arrival order while the next batch's
//     workspace (control words, descriptors, 4C low-res planes per request)
//     fits in a free range of the arena: admission by HBM footprint;
//   * launches each admitted group as one persistent batched kernel on the
//     next of its streams, so requests that arrive while earlier batches run
//     are admitted as memory frees up and their work overlaps on the device.
//     A request the batched kernels do not run (a low-res radius above their
//     limit, area subsampling, a colour guide) is admitted alone and runs
//     the per-image kernels.
// A request's result is exactly what the batched launch computes for it,
// whatever else shares its batch (tile shapes depend only on the radius).
#include <hip/hip_runtime_api.h>

#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "gf_api_internal.h"
#include "gf_batch_host.h"
#include "gf_range_alloc.h"

namespace gf {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

struct Request {
    uint64_t ticket;
    gf_image I, p, q;
    gf_params pr;
    size_t footprint;  // workspace bytes of this request alone
    int R;             // low-res radius (decides the request's tile height)
    bool solo;         // runs the per-image kernels, in a batch of its own
    gf_req_stats st{};
    gf_status status = GF_PENDING;
};

class Engine {
  public:
    Engine(gf_ctx *ctx, char *arena, size_t bytes, int max_inflight, std::vector<hipStream_t> streams,
           unsigned *err_slots)
        : ctx_(ctx), arena_(arena), bytes_(bytes), max_inflight_(max_inflight), streams_(streams),
          alloc_(bytes), err_slots_(err_slots) {
        for (int i = kMaxBatches - 1; i >= 0; --i) free_slots_.push_back(i);
        worker_ = std::thread([this] { run(); });
    }

    ~Engine() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        worker_.join();
        for (auto &b : inflight_) {
            (void)hipEventSynchronize(b.done);
            (void)hipEventDestroy(b.done);
        }
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        (void)hipFree(arena_);
        (void)hipHostFree(err_slots_);
    }

    gf_status submit(const gf_image *I, const gf_image *p, gf_image *q, const gf_params *pr,
                     uint64_t *ticket) {
        gf_status st = validate(I, p, q, pr);
        if (st != GF_OK) return st;
        BatchPlan one;
        if ((st = plan_batch(1, I, p, q, pr, nullptr, ctx_batch_cfg(ctx_), &one)) != GF_OK) return st;
        if (one.ws_bytes > bytes_)
            return fail(GF_ENOMEM, "request needs %zu bytes of arena, the arena holds %zu", one.ws_bytes,
                        bytes_);
        std::lock_guard<std::mutex> lk(mu_);
        if ((int)reqs_.size() >= max_inflight_)
            return fail(GF_EBUSY, "%d requests held (max_inflight)", (int)reqs_.size());
        const uint64_t t = next_ticket_++;
        Request &r = reqs_[t];
        r.ticket = t;
        r.I = *I;
        r.p = *p;
        r.q = *q;
        r.pr = *pr;
        r.footprint = one.ws_bytes;
        r.R = lowres_radius(pr->r, pr->s);
        r.solo = one.th == 0;
        r.st.t_submit = now_s();
        queue_.push_back(t);
        *ticket = t;
        cv_work_.notify_all();
        return GF_OK;
    }

    gf_status poll(uint64_t ticket, int32_t wait_ms, gf_req_stats *stats) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(GF_EINVAL, "unknown or retired ticket %llu", (unsigned long long)ticket);
        auto finished = [&] { return reqs_.at(ticket).status != GF_PENDING; };
        if (!finished() && wait_ms != 0) {
            if (wait_ms < 0) cv_done_.wait(lk, finished);
            else cv_done_.wait_for(lk, std::chrono::milliseconds(wait_ms), finished);
        }
        Request &r = reqs_.at(ticket);
        if (r.status == GF_PENDING)
            return wait_ms > 0 ? fail(GF_ETIMEDOUT, "request %llu still pending", (unsigned long long)ticket)
                               : GF_PENDING;
        const gf_status st = r.status;
        if (stats) *stats = r.st;
        reqs_.erase(ticket);
        cv_work_.notify_all();  // a held slot freed
        if (st != GF_OK) return fail(st, "request %llu failed on the device", (unsigned long long)ticket);
        return GF_OK;
    }

  private:
    struct Batch {
        std::vector<uint64_t> tickets;
        size_t off, bytes;
        hipEvent_t done;
        int slot;  // pinned slot receiving the batch's error word
    };

    void run() {
        (void)hipSetDevice(ctx_->device);
        // timed waits of this thread end within a microsecond of their
        // deadline (the default slack of 50 us would add to every request's
        // completion time)
        (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            retire();
            admit();
            if (stop_ && queue_.empty() && inflight_.empty()) break;
            // poll in-flight work often; otherwise sleep until a submit/poll wakes us
            if (!inflight_.empty()) cv_work_.wait_for(lk, std::chrono::microseconds(kPollUs));
            else cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
        }
    }

    // Finished batches: mark requests, free arena ranges.
    void retire() {
        bool any = false;
        for (size_t k = 0; k < inflight_.size();) {
            Batch &b = inflight_[k];
            const hipError_t e = hipEventQuery(b.done);
            if (e == hipErrorNotReady) {
                ++k;
                continue;
            }
            const double t = now_s();
            const bool bad = e != hipSuccess || err_slots_[b.slot] != 0;
            for (uint64_t tk : b.tickets) {
                auto it = reqs_.find(tk);
                if (it == reqs_.end()) continue;
                it->second.status = bad ? GF_EDEVICE : GF_OK;
                it->second.st.t_done = t;
            }
            (void)hipEventDestroy(b.done);
            free_slots_.push_back(b.slot);
            alloc_.release(b.off, b.bytes);
            inflight_.erase(inflight_.begin() + (long)k);
            any = true;
        }
        if (any) cv_done_.notify_all();
    }

    // Admit queued requests (arrival order) into one batch while the batch's
    // workspace fits in a free arena range, and launch it.  A batch holds
    // only requests that get the same tile heights on their own, so the
    // batch's tile heights are theirs and every result has the bits of the
    // request run alone, whatever it was batched with.
    void admit() {
        while (!queue_.empty() && !free_slots_.empty()) {
            const size_t room = alloc_.largest();
            const gf_batch_cfg cfg = ctx_batch_cfg(ctx_);
            std::vector<uint64_t> take;
            std::vector<gf_image> I, p, q;
            std::vector<gf_params> pr;
            size_t need = 0;
            int th = -1;
            for (uint64_t tk : queue_) {
                const Request &r = reqs_.at(tk);
                // a request for the per-image kernels goes alone (key -2); the
                // others join requests that get the same tile heights alone
                const TileCfg bt = batch_tiles(cfg, r.R);
                const int rth = r.solo ? -2 : bt.coeff_th * 256 + bt.box_th;
                if (th == -2 || (rth == -2 && th != -1)) break;
                if (th < 0) th = rth;
                // the batch's own workspace grows by this request's planes and descriptor
                const size_t grow = r.footprint;
                if (rth != th || need + grow > room || (int)take.size() >= kMaxBatch) break;
                need += grow;
                take.push_back(tk);
                I.push_back(r.I);
                p.push_back(r.p);
                q.push_back(r.q);
                pr.push_back(r.pr);
            }
            if (take.empty()) return;  // the head does not fit yet: wait for a batch to finish
            BatchPlan plan;
            if (plan_batch((int)take.size(), I.data(), p.data(), q.data(), pr.data(), nullptr, cfg, &plan) != GF_OK) {
                fail_requests(take);
                continue;
            }
            size_t off = 0;
            const size_t bytes = round256(plan.ws_bytes);
            if (!alloc_.alloc(bytes, &off)) return;  // cannot happen (need >= plan size), wait
            char *ws = arena_ + off;
            (void)plan_batch((int)take.size(), I.data(), p.data(), q.data(), pr.data(), ws, cfg, &plan);
            hipStream_t s = streams_[next_stream_++ % streams_.size()];
            Batch b{take, off, bytes, nullptr, free_slots_.back()};
            free_slots_.pop_back();
            err_slots_[b.slot] = 0;
            const double t = now_s();
            for (uint64_t tk : take) reqs_.at(tk).st.t_admit = t;
            gf_status st;
            if (plan.th == 0) {
                // per-image kernels on the request's share of the workspace; no error word
                const BDesc &d = plan.desc[0];
                st = run_fast(ctx_, &I[0], &p[0], &q[0], &pr[0], d.coef, workspace_bytes(d.g), s, nullptr);
            } else {
                st = launch_plan(ctx_, plan, ws, s);
            }
            hipError_t e = hipSuccess;
            if (st == GF_OK && plan.th == 0) {
                e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(b.done, s);
            } else if (st == GF_OK) {
                // the kernel's error word (control word 1) comes back with the batch
                e = hipMemcpyAsync(&err_slots_[b.slot], ws + sizeof(unsigned), sizeof(unsigned),
                                   hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(b.done, s);
            }
            const double t1 = now_s();
            for (uint64_t tk : take) reqs_.at(tk).st.t_start = t1;
            queue_.erase(queue_.begin(), queue_.begin() + (long)take.size());
            if (st != GF_OK || e != hipSuccess) {
                if (b.done) (void)hipEventDestroy(b.done);
                (void)hipStreamSynchronize(s);
                free_slots_.push_back(b.slot);
                alloc_.release(off, bytes);
                fail_requests(take);
                continue;
            }
            inflight_.push_back(b);
        }
    }

    void fail_requests(const std::vector<uint64_t> &take) {
        const double t = now_s();
        for (uint64_t tk : take) {
            auto it = reqs_.find(tk);
            if (it == reqs_.end()) continue;
            it->second.status = GF_EDEVICE;
            it->second.st.t_done = t;
        }
        auto end = queue_.end();
        for (uint64_t tk : take) end = std::remove(queue_.begin(), end, tk);
        queue_.erase(end, queue_.end());
        cv_done_.notify_all();
    }

  public:
    static constexpr int kMaxBatch = 64;     // requests per launch (bounds the latency of a batch)
    static constexpr int kPollUs = 20;       // completion polling period while batches are in flight
    static constexpr int kMaxBatches = 256;  // batches in flight (pinned error slots)

  private:

    gf_ctx *ctx_;
    char *arena_;
    size_t bytes_;
    int max_inflight_;
    std::vector<hipStream_t> streams_;
    size_t next_stream_ = 0;
    RangeAlloc alloc_;
    unsigned *err_slots_;            // pinned, kMaxBatches words
    std::vector<int> free_slots_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::map<uint64_t, Request> reqs_;  // held requests (queued, running or finished, not yet polled)
    std::deque<uint64_t> queue_;        // not yet admitted, arrival order
    std::vector<Batch> inflight_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    std::thread worker_;
};

static constexpr int kEngineStreams = 3;

gf_status engine_start(gf_ctx *ctx, size_t arena_bytes, int max_inflight) {
    char *arena = nullptr;
    hipError_t e = hipMalloc((void **)&arena, arena_bytes);
    if (e != hipSuccess) return fail(GF_ENOMEM, "arena hipMalloc(%zu): %s", arena_bytes, hipGetErrorString(e));
    std::vector<hipStream_t> streams;
    for (int i = 0; i < kEngineStreams; ++i) {
        hipStream_t s = nullptr;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
            for (hipStream_t t : streams) (void)hipStreamDestroy(t);
            (void)hipFree(arena);
            return fail(GF_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        streams.push_back(s);
    }
    unsigned *slots = nullptr;
    if ((e = hipHostMalloc((void **)&slots, sizeof(unsigned) * Engine::kMaxBatches, hipHostMallocDefault)) !=
        hipSuccess) {
        for (hipStream_t t : streams) (void)hipStreamDestroy(t);
        (void)hipFree(arena);
        return fail(GF_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    try {
        ctx->engine = new Engine(ctx, arena, arena_bytes, max_inflight, streams, slots);
    } catch (...) {
        for (hipStream_t t : streams) (void)hipStreamDestroy(t);
        (void)hipFree(arena);
        (void)hipHostFree(slots);
        return fail(GF_ENOMEM, "cannot start the request engine");
    }
    return GF_OK;
}

void engine_stop(gf_ctx *ctx) {
    delete ctx->engine;
    ctx->engine = nullptr;
}

}  // namespace gf

using namespace gf;

extern "C" {

gf_status gf_submit(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q, const gf_params *pr,
                    uint64_t *ticket) {
    if (!ctx) return fail(GF_EINVAL, "gf_submit needs a context");
    if (!ticket) return fail(GF_EINVAL, "ticket is NULL");
    if (!ctx->engine) return fail(GF_EINVAL, "context was created without a request arena");
    return ctx->engine->submit(I, p, q, pr, ticket);
}

gf_status gf_poll(gf_ctx *ctx, uint64_t ticket, int32_t wait_ms, gf_req_stats *stats) {
    if (!ctx) return fail(GF_EINVAL, "gf_poll needs a context");
    if (!ctx->engine) return fail(GF_EINVAL, "context was created without a request arena");
    return ctx->engine->poll(ticket, wait_ms, stats);
}

}  // extern "C"
