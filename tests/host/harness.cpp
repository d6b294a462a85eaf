// Host-code checks of libgf.so under sanitizers (built and run by
// tests/test_host_sanitizers.py against the stand-in runtime of
// fake_hip.cpp; no GPU).  Each check prints its name; any failure prints a
// message and exits with status 1.  Sanitizer reports end the run with
// their own status.
//
//   validation  invalid calls rejected on the host, with messages
//   range       the request arena's first-fit range allocator against a
//               byte map, over random allocate / release sequences
//   plan        batch plans: queue bases, phase counts and workspace layout
//               of random batches
//   tuning      tuning files written and read back; malformed files refused
//   engine      gf_submit / gf_poll from several threads at once, with
//               batches that fail (error word set) among them
//   calls       gf_fast / gf_plain / batched calls with context workspaces,
//               profiling and the autotuners
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "gf.h"
#include "gf_api_internal.h"
#include "gf_batch_host.h"
#include "gf_range_alloc.h"

extern std::atomic<int> fake_fail_next;
size_t fake_live_allocations();

#define CHECK(cond, ...)                                                      \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "%s:%d: check failed: %s: ", __FILE__, __LINE__, #cond); \
            fprintf(stderr, __VA_ARGS__);                                     \
            fprintf(stderr, " (last error: %s)\n", gf_last_error(nullptr));   \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

// Fake device addresses: never dereferenced by the host code under test.
static std::atomic<uintptr_t> g_next_addr{0x100000000ull};
static void *fake_buffer(size_t bytes) {
    return (void *)g_next_addr.fetch_add((bytes + 4095) / 4096 * 4096 + 4096);
}

static gf_image image(int c, int h, int w, gf_dtype dt = GF_F16) {
    gf_image im{};
    im.dtype = dt;
    im.c = c;
    im.h = h;
    im.w = w;
    im.row_stride = w;
    im.plane_stride = (int64_t)h * w;
    im.data = fake_buffer((size_t)c * h * w * (dt == GF_F32 ? 4 : 2));
    return im;
}

static gf_params params(int r, int s, double eps = 1e-3, gf_subsample sub = GF_SUB_NEAREST,
                        gf_border b = GF_BORDER_CLIP) {
    gf_params p{};
    p.r = r;
    p.s = s;
    p.eps = eps;
    p.sub = sub;
    p.border = b;
    return p;
}

// ---------------------------------------------------------------- validation

static void check_validation() {
    gf_image I = image(1, 64, 80, GF_F32), p = image(3, 64, 80, GF_F32), q = image(3, 64, 80, GF_F32);
    gf_params pr = params(8, 4, 1e-2);
    void *ws = fake_buffer(1 << 20);
    auto call = [&](gf_image a, gf_image b, gf_image c, gf_params d, size_t wsb = 1 << 20) {
        return gf_fast(nullptr, &a, &b, &c, &d, ws, wsb, nullptr);
    };
    gf_image bad = I;
    bad.data = nullptr;
    CHECK(call(bad, p, q, pr) == GF_EINVAL, "null data");
    CHECK(strlen(gf_last_error(nullptr)) > 0, "a message is set");
    bad = p;
    bad.c = 2;
    CHECK(call(I, bad, q, pr) == GF_EINVAL, "channel mismatch");
    bad = I;
    bad.c = 2;
    CHECK(call(bad, p, q, pr) == GF_ENOTSUP, "two-channel guide");
    gf_params bp = pr;
    bp.eps = 0.0;
    CHECK(call(I, p, q, bp) == GF_EINVAL, "eps 0");
    bp = pr;
    bp.s = 0;
    CHECK(call(I, p, q, bp) == GF_EINVAL, "s 0");
    bp = pr;
    bp.r = 100000;
    CHECK(call(I, p, q, bp) == GF_ENOTSUP, "radius");
    gf_image alias = q;
    alias.data = p.data;
    CHECK(call(I, p, alias, pr) == GF_EINVAL, "q aliases p");
    CHECK(call(I, p, q, pr, 16) == GF_ENOMEM, "workspace too small");
    CHECK(gf_fast(nullptr, &I, &p, &q, &pr, nullptr, 0, nullptr) == GF_EINVAL, "no workspace, no context");
    CHECK(gf_submit(nullptr, &I, &p, &q, &pr, nullptr) == GF_EINVAL, "submit without context");
    CHECK(gf_workspace_bytes(0, 10, 1, &pr) == 0, "empty image");
    CHECK(gf_workspace_bytes(64, 80, 3, &pr) > 0, "workspace size");
}

// ---------------------------------------------------------------- range allocator

static void check_range() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 20; ++trial) {
        const size_t size = 1024 + rng() % 16000;
        gf::RangeAlloc ra(size);
        std::vector<int> owner(size, -1);  // byte map: which allocation holds each byte
        struct Live {
            size_t off, n;
        };
        std::vector<Live> live;
        for (int step = 0; step < 600; ++step) {
            if (live.empty() || rng() % 3) {
                const size_t n = 1 + rng() % (size / 8);
                size_t off = 0;
                // the model: is there a free run of n bytes, and which is the largest?
                size_t largest = 0, run = 0;
                for (size_t b = 0; b < size; ++b) {
                    run = owner[b] < 0 ? run + 1 : 0;
                    largest = std::max(largest, run);
                }
                CHECK(ra.largest() == largest, "largest %zu, model %zu", ra.largest(), largest);
                const bool ok = ra.alloc(n, &off);
                CHECK(ok == (largest >= n), "alloc(%zu) = %d with largest free run %zu", n, ok, largest);
                if (!ok) continue;
                CHECK(off + n <= size, "range [%zu, %zu) past the arena", off, off + n);
                // first fit: no free run of n bytes starts before off
                run = 0;
                for (size_t b = 0; b < off; ++b) {
                    run = owner[b] < 0 ? run + 1 : 0;
                    CHECK(run < n, "first fit: a run of %zu bytes ends at %zu before %zu", n, b, off);
                }
                for (size_t b = off; b < off + n; ++b) {
                    CHECK(owner[b] < 0, "byte %zu given twice", b);
                    owner[b] = (int)live.size();
                }
                live.push_back({off, n});
            } else {
                const size_t k = rng() % live.size();
                ra.release(live[k].off, live[k].n);
                for (size_t b = live[k].off; b < live[k].off + live[k].n; ++b) owner[b] = -1;
                live[k] = live.back();
                live.pop_back();
                for (size_t j = 0; j < live.size(); ++j)  // renumber owners
                    for (size_t b = live[j].off; b < live[j].off + live[j].n; ++b) owner[b] = (int)j;
            }
        }
        for (auto &l : live) ra.release(l.off, l.n);
        CHECK(ra.largest() == size, "everything released coalesces back to one range");
    }
}

// ---------------------------------------------------------------- batch plans

static void check_plan() {
    std::mt19937_64 rng(11);
    for (int trial = 0; trial < 200; ++trial) {
        const int n = 1 + (int)(rng() % 40);
        std::vector<gf_image> I, p, q;
        std::vector<gf_params> pr;
        for (int i = 0; i < n; ++i) {
            const int h = 1 + (int)(rng() % 900), w = 1 + (int)(rng() % 1300), c = 1 + (int)(rng() % 4);
            const int s = (int[]){1, 2, 3, 4, 8}[rng() % 5];
            I.push_back(image(1, h, w));
            p.push_back(image(c, h, w));
            q.push_back(image(c, h, w));
            pr.push_back(params((int)(rng() % 40), s, 1e-3, rng() % 2 ? GF_SUB_NEAREST : GF_SUB_BILINEAR,
                                (gf_border)(rng() % 3)));
        }
        const gf_batch_cfg cfg{(int32_t)(rng() % 2), (int32_t[]){0, 8, 16, 24}[rng() % 4]};
        gf::BatchPlan plan;
        char *base = (char *)fake_buffer(1 << 20);
        const gf_status st = gf::plan_batch(n, I.data(), p.data(), q.data(), pr.data(), base, cfg, &plan);
        CHECK(st == GF_OK, "plan of %d images", n);
        CHECK(plan.ws_bytes == gf_batched_workspace_bytes(n, I.data(), p.data(), pr.data()),
              "plan %zu bytes, gf_batched_workspace_bytes %zu", plan.ws_bytes,
              gf_batched_workspace_bytes(n, I.data(), p.data(), pr.data()));
        std::vector<int> seen(n, 0);
        unsigned next[3] = {0, plan.p1, plan.p2};
        char *lo = base + plan.desc_off + sizeof(gf::BDesc) * n;
        int last_class = -1;
        for (int k = 0; k < n; ++k) {
            const gf::BDesc &d = plan.desc[k];
            const int i = plan.order[k];
            CHECK(i >= 0 && i < n && !seen[i]++, "order is a permutation");
            const int cls = gf::ratio_class(pr[i].s);
            CHECK(cls >= last_class, "images sorted by ratio class");
            last_class = cls;
            for (int ph = 0; ph < 3; ++ph) {
                CHECK(d.base[ph] == next[ph], "queue base of image %d phase %d", k, ph);
                next[ph] += d.ntiles[ph];
            }
            const char *c0 = (const char *)d.coef;
            const size_t bytes = gf::workspace_bytes(d.g);
            CHECK(c0 >= lo && c0 + bytes <= base + plan.ws_bytes, "image %d planes inside the workspace", k);
            CHECK(((uintptr_t)c0 % 256) == 0, "planes 256-byte aligned");
            lo = (char *)c0 + bytes;
            CHECK(d.mean == d.coef + (size_t)d.g.lps * 2 * d.g.C, "box means after a, b");
        }
        CHECK(next[0] == plan.p1 && next[1] == plan.p2 && next[2] == plan.total, "phase ends");
    }
}

// ---------------------------------------------------------------- tuning files

static std::string tmpfile_path(const char *tag) {
    char buf[256];
    snprintf(buf, sizeof buf, "/tmp/gf_host_check_%d_%s.json", (int)getpid(), tag);
    return buf;
}

static void write_file(const std::string &path, const char *text) {
    FILE *f = fopen(path.c_str(), "w");
    CHECK(f != nullptr, "open %s", path.c_str());
    fputs(text, f);
    fclose(f);
}

static std::string read_file(const std::string &path) {
    std::string s;
    FILE *f = fopen(path.c_str(), "r");
    CHECK(f != nullptr, "open %s", path.c_str());
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    fclose(f);
    return s;
}

static void check_tuning() {
    gf_ctx *a = nullptr, *b = nullptr;
    CHECK(gf_ctx_create(&a, 0, 0, 0) == GF_OK, "ctx");
    CHECK(gf_ctx_create(&b, 0, 0, 0) == GF_OK, "ctx");
    gf_tiles t{24, 48};
    gf_params pr = params(16, 4);
    CHECK(gf_ctx_set_tiles(a, GF_F32, 3000, 4000, 3, &pr, &t) == GF_OK, "pin");
    t = gf_tiles{16, 24};
    pr = params(8, 2);
    CHECK(gf_ctx_set_tiles(a, GF_F16, 1000, 1000, 1, &pr, &t) == GF_OK, "pin");
    const std::string p1 = tmpfile_path("a"), p2 = tmpfile_path("b");
    CHECK(gf_ctx_save_tuning(a, p1.c_str()) == GF_OK, "save");
    CHECK(gf_ctx_load_tuning(b, p1.c_str()) == GF_OK, "load");
    CHECK(gf_ctx_save_tuning(b, p2.c_str()) == GF_OK, "save");
    CHECK(read_file(p1) == read_file(p2), "a file read back and written again is the same");
    // malformed or hostile files: refused or ignored, never a crash
    const char *bad[] = {
        "", "garbage", "{\"entries\": [\n{\"key\": }\n]}\n", "{\"key\": 1, \"coeff_th\": 8}\n",
        "{\"key\": 99999999999999999999999999, \"coeff_th\": 8, \"box_th\": 8}\n",
        "{\"key\": 5, \"coeff_th\": -2147483648, \"box_th\": 7}\n",
    };
    for (const char *text : bad) {
        write_file(p2, text);
        (void)gf_ctx_load_tuning(b, p2.c_str());
    }
    std::string longline = "{\"key\": 1, \"coeff_th\": 8, \"box_th\": 8}";
    longline.append(5000, ' ');
    write_file(p2, (longline + "\n").c_str());
    (void)gf_ctx_load_tuning(b, p2.c_str());
    CHECK(gf_ctx_load_tuning(b, "/nonexistent/dir/x.json") == GF_EINVAL, "missing file");
    CHECK(gf_ctx_save_tuning(b, "/nonexistent/dir/x.json") == GF_EINVAL, "unwritable file");
    // a call after loading odd tiles still runs (unfit tiles fall back to the built-in choice)
    gf_image I = image(1, 300, 400), p = image(3, 300, 400), q = image(3, 300, 400);
    pr = params(8, 4);
    CHECK(gf_fast(b, &I, &p, &q, &pr, nullptr, 0, nullptr) == GF_OK, "call with loaded tiles");
    unlink(p1.c_str());
    unlink(p2.c_str());
    gf_ctx_destroy(a);
    gf_ctx_destroy(b);
}

// ---------------------------------------------------------------- request engine

static void check_engine(int threads, int per_thread) {
    gf_ctx *ctx = nullptr;
    CHECK(gf_ctx_create(&ctx, 0, (size_t)64 << 20, 256) == GF_OK, "ctx with arena");
    // too large to ever fit the arena
    {
        gf_image I = image(1, 8000, 8000), p = image(3, 8000, 8000), q = image(3, 8000, 8000);
        gf_params pr = params(4, 1);
        uint64_t t = 0;
        CHECK(gf_submit(ctx, &I, &p, &q, &pr, &t) == GF_ENOMEM, "request above the arena");
    }
    std::atomic<int> ok{0}, failed{0};
    fake_fail_next = 3;  // three batches come back with their error word set
    auto worker = [&](int id) {
        std::mt19937_64 rng(100 + id);
        std::vector<uint64_t> mine;
        std::vector<bool> retired;
        auto count = [&](gf_status st, const gf_req_stats &s) {
            CHECK(st == GF_OK || st == GF_EDEVICE, "poll status %d", (int)st);
            if (st == GF_OK) {
                CHECK(s.t_submit <= s.t_admit && s.t_admit <= s.t_start && s.t_start <= s.t_done, "stamps");
                ++ok;
            } else {
                ++failed;
            }
        };
        for (int k = 0; k < per_thread; ++k) {
            const int h = 16 + (int)(rng() % 600), w = 16 + (int)(rng() % 800), c = 1 + (int)(rng() % 3);
            gf_image I = image(1, h, w), p = image(c, h, w), q = image(c, h, w);
            gf_params pr = params((int)(rng() % 24), (int[]){1, 2, 4, 8}[rng() % 4], 1e-3,
                                  rng() % 5 ? GF_SUB_NEAREST : GF_SUB_AREA);
            uint64_t t = 0;
            gf_status st;
            while ((st = gf_submit(ctx, &I, &p, &q, &pr, &t)) == GF_EBUSY) std::this_thread::yield();
            CHECK(st == GF_OK, "submit");
            mine.push_back(t);
            retired.push_back(false);
            if (rng() % 4 == 0) {  // poll an earlier one without waiting
                const size_t j = rng() % mine.size();
                gf_req_stats s{};
                if (!retired[j]) {
                    const gf_status st = gf_poll(ctx, mine[j], 0, &s);
                    if (st != GF_PENDING) {
                        count(st, s);
                        retired[j] = true;
                    }
                }
            }
        }
        for (size_t j = 0; j < mine.size(); ++j) {
            if (retired[j]) continue;
            gf_req_stats s{};
            count(gf_poll(ctx, mine[j], -1, &s), s);
            CHECK(gf_poll(ctx, mine[j], 0, nullptr) == GF_EINVAL, "a retired ticket");
        }
    };
    std::vector<std::thread> ts;
    for (int i = 0; i < threads; ++i) ts.emplace_back(worker, i);
    for (auto &t : ts) t.join();
    CHECK(failed.load() >= 1, "requests of the failed batches report GF_EDEVICE (%d failed)", failed.load());
    fprintf(stderr, "engine: %d ok, %d failed\n", ok.load(), failed.load());
    gf_ctx_destroy(ctx);
    fake_fail_next = 0;
}

// ---------------------------------------------------------------- other calls

static void check_calls() {
    gf_ctx *ctx = nullptr;
    CHECK(gf_ctx_create(&ctx, 0, 0, 0) == GF_OK, "ctx");
    CHECK(gf_ctx_profile(ctx, 1) == GF_OK, "profile on");
    for (int k = 0; k < 3; ++k) {  // the context's workspace grows
        const int h = 200 * (k + 1), w = 300 * (k + 1);
        gf_image I = image(1, h, w, GF_F32), p = image(3, h, w, GF_F32), q = image(3, h, w, GF_F32);
        gf_params pr = params(8, k + 1, 1e-2, k == 2 ? GF_SUB_AREA : GF_SUB_NEAREST, GF_BORDER_REFLECT101);
        CHECK(gf_fast(ctx, &I, &p, &q, &pr, nullptr, 0, nullptr) == GF_OK, "gf_fast");
        CHECK(gf_plain(ctx, &I, &p, &q, 4, 1e-2, GF_BORDER_CLIP, nullptr, 0, nullptr) == GF_OK, "gf_plain");
        CHECK(gf_detail_enhance(ctx, &I, &p, &q, &pr, 5.0, nullptr, 0, nullptr) == GF_OK, "detail");
        gf_image Ic = image(3, h, w, GF_F32);
        CHECK(gf_fast(ctx, &Ic, &p, &q, &pr, nullptr, 0, nullptr) == GF_OK, "colour guide");
    }
    gf_kernel_time kt[GF_NKERNELS];
    CHECK(gf_ctx_profile_read(ctx, kt) == GF_OK, "profile read");
    CHECK(kt[GF_K_OUTPUT].launches >= 3, "output launches timed");
    gf_ctx_profile(ctx, 0);
    // the tile autotuner
    gf_image I = image(1, 500, 700), p = image(2, 500, 700), q = image(2, 500, 700);
    gf_params pr = params(16, 4);
    gf_tiles best{};
    gf_tune_result res[64];
    int32_t nres = 0;
    void *ws = fake_buffer(64 << 20);
    CHECK(gf_tune(ctx, &I, &p, &q, &pr, ws, 64 << 20, nullptr, 2, &best, res, 64, &nres) == GF_OK, "gf_tune");
    CHECK(nres > 0, "tuner results");
    // batches: eager, prepared, tuned
    std::vector<gf_image> Is, ps, qs;
    std::vector<gf_params> prs;
    for (int i = 0; i < 6; ++i) {
        Is.push_back(image(1, 100 + 50 * i, 200 + 30 * i));
        ps.push_back(image(1 + i % 3, 100 + 50 * i, 200 + 30 * i));
        qs.push_back(image(1 + i % 3, 100 + 50 * i, 200 + 30 * i));
        prs.push_back(params(4 + i, 1 + i % 4));
    }
    CHECK(gf_fast_batched(ctx, 6, Is.data(), ps.data(), qs.data(), prs.data(), nullptr, 0, nullptr) == GF_OK,
          "batched");
    const size_t wsb = gf_batched_workspace_bytes(6, Is.data(), ps.data(), prs.data());
    void *bws = nullptr;
    CHECK(hipMalloc(&bws, wsb) == hipSuccess, "batch workspace");
    gf_batch *b = nullptr;
    CHECK(gf_batch_create(ctx, 6, Is.data(), ps.data(), qs.data(), prs.data(), bws, wsb, nullptr, &b) == GF_OK,
          "batch create");
    CHECK(gf_batch_launch(b, nullptr) == GF_OK, "batch launch");
    gf_batch_destroy(b);
    gf_batch_cfg cfg{};
    gf_batch_tune_result bres[16];
    int32_t nb = 0;
    CHECK(gf_tune_batched(ctx, 6, Is.data(), ps.data(), qs.data(), prs.data(), bws, wsb, nullptr, 2, &cfg, bres,
                          16, &nb) == GF_OK,
          "batch tuner");
    CHECK(nb > 0, "batch tuner results");
    CHECK(gf_ctx_set_wait_limit(ctx, 0) == GF_OK && gf_ctx_set_wait_limit(ctx, -1) == GF_OK, "wait limit");
    CHECK(gf_ctx_set_wait_limit(ctx, (int64_t)1 << 40) == GF_EINVAL, "wait limit range");
    (void)hipFree(bws);
    gf_ctx_destroy(ctx);
}

int main(int argc, char **argv) {
    const std::string only = argc > 1 ? argv[1] : "";
    auto run = [&](const char *name, auto fn) {
        if (!only.empty() && only != name) return;
        fprintf(stderr, "check: %s\n", name);
        fn();
    };
    run("validation", check_validation);
    run("range", check_range);
    run("plan", check_plan);
    run("tuning", check_tuning);
    run("engine", [] { check_engine(4, 60); });
    run("calls", check_calls);
    CHECK(fake_live_allocations() == 0, "%zu device or pinned allocations left", fake_live_allocations());
    fprintf(stderr, "host checks passed\n");
    return 0;
}
