/*
 * gf.h - C ABI of the MI355X (gfx950) guided-filter library, libgf.so.
 *
 * Implements the guided filter and the Fast Guided Filter of
 * K. He and J. Sun, "Fast Guided Filter", arXiv 1505.00996:
 *   - gf_plain : Algorithm 1 (Eqs. 2-4): four box means of I, p, I*I, I*p at
 *                radius r, the coefficients a = cov(I,p)/(var(I)+eps) and
 *                b = mean(p) - a mean(I), their box means, q = mean_a*I + mean_b.
 *   - gf_fast  : Algorithm 2: the same steps on I and p subsampled by s at
 *                radius r/s, with mean_a and mean_b bilinearly upsampled and
 *                applied to the full-resolution guide I (Sec. 2).
 *   - gf_fast_batched : Algorithm 2 for many images of different sizes in one
 *                launch.
 *   - gf_submit / gf_poll : an asynchronous request interface that batches the
 *                requests in flight (same result as gf_fast per request).
 *
 * Conventions (where the paper leaves a choice):
 *   - window of radius r = (2r+1)x(2r+1) square; box means are taken over the
 *     part of the window inside the image and divided by its pixel count
 *     (GF_BORDER_CLIP), which makes Eq. 4's "average over the windows that
 *     contain pixel i" a box mean;
 *   - variance is the population variance mean(I*I) - mean(I)^2, clamped at 0;
 *   - r' = r/s rounded half up, at least 1 when r > 0;
 *   - the low-resolution maps are ceil(h/s) x ceil(w/s);
 *   - GF_SUB_NEAREST takes full-res pixel s*y + floor(s/2) (clamped);
 *     GF_SUB_BILINEAR samples the low-res pixel centre s*y + (s-1)/2 with two
 *     clamped taps per axis (no antialias prefilter);
 *   - upsampling is bilinear with half-pixel centres, u = (y+0.5)/s - 0.5,
 *     taps clamped to the low-res map;
 *   - a multi-channel p is filtered channel by channel with the same gray I.
 *
 * Colour guide (I with 3 channels; the paper counts channels as a cost
 * factor and takes the colour form of the guided filter from its earlier
 * definition): per window q = a.I + b with a a 3-vector,
 * a = (Sigma + eps U)^-1 (mean(I p) - mean(I) mean(p)), b = mean(p) - a.mean(I),
 * Sigma the 3x3 population covariance of I in the window (sums in FP64, the
 * 3x3 solve in FP64), and q = mean_a.I + mean_b.  gf_plain, gf_fast,
 * gf_joint_upsample, gf_detail_enhance and the batched and prepared-batch
 * calls take it (a batch holding one runs image by image, and gf_submit
 * runs such a request in a batch of its own); gf_tune refuses it
 * (GF_ENOTSUP), as every call does a low-res radius whose colour tiles do
 * not fit in LDS (above about 24).
 *
 * Options for the conventions of other image libraries (gf_params):
 *   - GF_BORDER_REPLICATE / GF_BORDER_REFLECT101: every box mean (of the
 *     statistics and of a, b) reads the map extended past its edges, by
 *     repeating the edge pixel or by mirroring about it without repeating it
 *     (... 2 1 | 0 1 ... n-1 | n-2 ..., repeated for windows wider than the
 *     map), and divides by (2r+1)^2.  Upsampling still clamps its taps;
 *   - GF_SUB_AREA: the low-res pixel (y, x) is the mean of the full-res
 *     block [s*y, s*y+s) x [s*x, s*x+s) clipped to the image.  It reads all
 *     of I and p, in a pass of its own (FP64 block sums, the mean stored as
 *     FP32 in the workspace); batched launches of a batch that holds such an
 *     image run image by image, and gf_submit runs such a request alone.
 *
 * Arithmetic: all window sums, coefficients and interpolation in FP32
 * (window sums of mean-shifted values, tile by tile); images may be stored as
 * FP32, FP16 or BF16, and 16-bit outputs are rounded to nearest even.
 *
 * Memory and ownership: every image pointer is DEVICE memory owned by the
 * caller, which keeps it alive and unmodified until the work has completed
 * (stream order for gf_plain/gf_fast/gf_fast_batched; a terminal gf_poll for
 * gf_submit).  The library only owns workspace: either the caller passes one
 * (device memory of at least the size the *_workspace_bytes call returns) or,
 * with workspace == NULL, the context's own buffer is used.  Calls that share
 * one context's buffer must not overlap on different streams.
 *
 * Errors: status codes only.  Arguments are validated on the host before any
 * HIP call; an invalid call returns GF_EINVAL (or GF_ENOTSUP) and launches
 * nothing.  gf_last_error() returns a message for the last failing call on
 * the calling thread.  Launch failures return GF_EDEVICE; faults inside a
 * kernel surface at the next synchronisation of the stream.
 *
 * Every entry point may be called with ctx == NULL except gf_submit and
 * gf_poll; it then runs on the current HIP device and needs an explicit
 * workspace.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GF_OK = 0,
    GF_PENDING = 1,     /* gf_poll: the request has not finished yet */
    GF_EINVAL = -1,     /* invalid argument, shape, stride, aliasing or ticket */
    GF_ENOMEM = -2,     /* workspace too small, or the request can never fit the arena */
    GF_EBUSY = -3,      /* request queue full; try again after polling */
    GF_ENOTSUP = -4,    /* valid but unsupported option (colour guide, radius too large) */
    GF_EDEVICE = -5,    /* a HIP call failed */
    GF_ETIMEDOUT = -6   /* gf_poll: wait time elapsed */
} gf_status;

typedef enum { GF_F32 = 0, GF_F16 = 1, GF_BF16 = 2 } gf_dtype;

typedef enum {
    GF_BORDER_CLIP = 0,       /* window clipped to the image, mean over in-image pixels */
    GF_BORDER_REPLICATE = 1,  /* image extended by its edge pixels, mean over (2r+1)^2 */
    GF_BORDER_REFLECT101 = 2  /* image mirrored about its edge pixels, mean over (2r+1)^2 */
} gf_border;

typedef enum { GF_SUB_NEAREST = 0, GF_SUB_BILINEAR = 1, GF_SUB_AREA = 2 } gf_subsample;

/*
 * A c x h x w image in device memory.  Element (k, y, x) is at
 * data + k*plane_stride + y*row_stride + x, strides counted in ELEMENTS.
 * Requirements: c >= 1, h >= 1, w >= 1, row_stride >= w,
 * plane_stride >= h*row_stride when c > 1.  For I, c is 1 (gray) or 3
 * (colour guide).  Any stride works; outputs whose rows start at multiples of
 * 64 bytes (row_stride * element size a multiple of 64, data aligned) are
 * written fastest: 6000 x 4000 fp16 RGB q with 12000-byte rows took the
 * output pass 38.4 us, with 12032- or 12288-byte rows 35.4-36.2 us.
 */
typedef struct {
    void *data;
    gf_dtype dtype;
    int32_t c, h, w;
    int64_t row_stride;
    int64_t plane_stride;
} gf_image;

/* Filter parameters: full-resolution radius r >= 0, subsampling ratio
 * s >= 1 (s = 1 is Algorithm 1), regulariser eps > 0 and finite (in units of
 * I^2), border convention, subsampling kind. */
typedef struct {
    int32_t r;
    int32_t s;
    double eps;
    gf_border border;
    gf_subsample sub;
} gf_params;

/* Per-request timestamps (seconds on the host's monotonic clock). */
typedef struct {
    double t_submit;  /* gf_submit accepted the request */
    double t_admit;   /* workspace reserved and work queued for launch */
    double t_start;   /* the launch carrying the request was issued */
    double t_done;    /* completion observed by the library */
} gf_req_stats;

typedef struct gf_ctx gf_ctx;

/* Create a context on HIP device `device`.  `arena_bytes` of device memory
 * are reserved for requests of gf_submit (0 = no request interface);
 * `max_inflight` bounds the requests held at once (queued or running).
 * Ownership: the context is released with gf_ctx_destroy, which waits for
 * the work it launched. */
gf_status gf_ctx_create(gf_ctx **out, int device, size_t arena_bytes, int max_inflight);
void gf_ctx_destroy(gf_ctx *ctx);

/* Message of the last failing call on this thread (never NULL). */
const char *gf_last_error(const gf_ctx *ctx);

/* Device workspace (bytes) gf_fast needs for an h x w image with c channels
 * of p and a gray guide: 4c low-resolution FP32 maps (a, b and their box
 * means), plus 1 + c with area subsampling.  Returns 0 for invalid
 * arguments. */
size_t gf_workspace_bytes(int32_t h, int32_t w, int32_t c, const gf_params *params);

/* The same for a guide of guide_c channels (1 or 3): a colour guide needs 8c
 * maps (a_0, a_1, a_2, b and their box means), plus 3 + c with area
 * subsampling. */
size_t gf_workspace_bytes_guide(int32_t h, int32_t w, int32_t guide_c, int32_t c, const gf_params *params);

/*
 * Algorithm 1 (guided filter) at full resolution: q = mean_a .* I + mean_b.
 * I: 1 x h x w (or 3 x h x w, colour guide); p, q: c x h x w; all three of one dtype; q must not overlap
 * I or p.  Enqueued on `hip_stream` (a hipStream_t; NULL = default stream);
 * returns after enqueue.  workspace: device memory of at least
 * gf_workspace_bytes(h, w, c, {r, 1, eps}) bytes, or NULL for the context's.
 */
gf_status gf_plain(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                   int32_t r, double eps, gf_border border,
                   void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * Algorithm 2 (Fast Guided Filter): subsample I and p by params->s, solve
 * Eqs. 2-3 and smooth a, b at radius r' = r/s on the low-resolution maps,
 * upsample mean_a, mean_b bilinearly and output q = mean_a .* I + mean_b
 * against the full-resolution I.  Same shapes, ownership and stream rules as
 * gf_plain.  With params->s == 1 it is gf_plain.  Independent images on
 * separate streams (each with its own context and workspace) overlap on
 * the GPU: one image's low-resolution passes run beside another's output
 * pass.  The output pass reserves 48 KB of LDS per workgroup it does not use
 * (at most three of its workgroups per CU), which kernels running beside it
 * on other streams share.
 */
gf_status gf_fast(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                  const gf_params *params, void *workspace, size_t workspace_bytes,
                  void *hip_stream);

/*
 * gf_fast for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  Same
 * arguments, shapes, result (bit for bit, with the same tiles) and stream
 * rules as gf_fast, without a workspace: the low-resolution maps go to a
 * fixed array of GF_NOALLOC_MAX_BYTES in device memory, one per GPU, held
 * until the process ends.  A call whose maps need more
 * (gf_workspace_bytes_guide(...) > GF_NOALLOC_MAX_BYTES) returns GF_ENOMEM
 * before any HIP call.  The call allocates nothing; the array's device
 * address is looked up once per device, at gf_ctx_create for the context's
 * device, else on the first call with that device current (make that first
 * call, or create the context, outside graph capture).  ctx may be NULL (the
 * current device, built-in tiles); with a context its device and tuned tiles
 * are used, but not its profiling.  Every call on one GPU shares that GPU's
 * array, and nothing in it needs clearing between calls; calls that overlap
 * on one GPU (on different streams or threads, or replays of graphs that
 * hold such calls) race on it and must be ordered by the caller.
 */
#define GF_NOALLOC_MAX_BYTES ((size_t)64 << 20)
gf_status gf_fast_noalloc(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                          const gf_params *params, void *hip_stream);

/*
 * Admission unit of the request interface: the bytes of the context's arena
 * one request of this shape occupies while it is in flight (its low-res maps
 * and its share of the batch's control words and descriptor table).
 * gf_submit refuses a request whose footprint exceeds the arena (GF_ENOMEM).
 * The dtype does not change it (all maps are FP32).  Gray guide (a colour
 * guide needs twice the maps).  0 for invalid sizes.
 */
size_t gf_footprint_bytes(int32_t h, int32_t w, int32_t c, gf_dtype dtype, const gf_params *params);

/*
 * Joint upsampling: the input arrives at low resolution and only the guide is
 * subsampled (the paper's introduction names joint upsampling as where this
 * subsampling first appeared).  I: 1 x h x w; p_low: c x ceil(h/s) x
 * ceil(w/s); q: c x h x w; one dtype.  Algorithm 2 runs with p' = p_low:
 * I' = subsample(I, s), a and b of Eqs. 2-3 at r' = r/s, their box means,
 * bilinear upsampling and q = mean_a .* I + mean_b on the full-resolution I.
 * The full-resolution p is never read.  With p_low the nearest subsample of
 * a full-resolution p, q equals gf_fast(I, p) bit for bit.  Workspace,
 * streams and errors as gf_fast (gf_workspace_bytes(h, w, c, params)).
 */
gf_status gf_joint_upsample(gf_ctx *ctx, const gf_image *I, const gf_image *p_low, gf_image *q,
                            const gf_params *params, void *workspace, size_t workspace_bytes,
                            void *hip_stream);

/*
 * Detail enhancement (the paper's first application): the filter output q of
 * gf_fast (gf_plain at s = 1) is the base layer and p - q the detail layer;
 * e = q + gain * (p - q) is written to `e` (c x h x w, like q) in place of q.
 * The paper's example amplifies the detail five times (gain 5).  q stays in
 * FP32 registers; e is formed with one FMA and rounded once for storage.  The
 * output pass also reads p (e * c bytes per pixel more than gf_fast).  gain
 * must be finite (GF_EINVAL); otherwise as gf_fast.
 */
gf_status gf_detail_enhance(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *e,
                            const gf_params *params, double gain, void *workspace,
                            size_t workspace_bytes, void *hip_stream);

/* Workspace (bytes) of gf_fast_batched for n images (device memory). */
size_t gf_batched_workspace_bytes(int32_t n, const gf_image *I, const gf_image *p,
                                  const gf_params *params);

/*
 * Algorithm 2 for n independent images (arrays of n descriptors and n
 * parameter sets; sizes, c, r, s and eps may differ, the dtype may not) in
 * one batched launch with the context's batch configuration (see
 * gf_batch_cfg; without a context the default).  Each q[k] equals what
 * gf_fast writes for image k with the batch's tiles ({tile_h, box tile
 * height}, see gf_batch_cfg).  Descriptor arrays are host memory, read
 * during the call.  workspace: at least gf_batched_workspace_bytes(...) of device memory,
 * or NULL for the context's.  Its first two uint32 words are the queue head
 * and an error word: once the launch has completed, a nonzero error word
 * means some tile stopped waiting for the previous phase of its image after
 * a bounded spin (about three seconds) and that image's q is incomplete.
 */
gf_status gf_fast_batched(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p,
                          gf_image *q, const gf_params *params,
                          void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * Schedules of a batched launch.  Both give every image the bits gf_fast
 * gives it with the batch's tiles: {tile_h, 48} under GF_BATCH_PHASES where
 * 48-row box tiles fit, else {tile_h, tile_h}.
 *   GF_BATCH_PHASES: one grid per phase (coefficient tiles, box-mean tiles,
 *     output blocks) over the tiles of all images: three kernel launches per
 *     batch, each at its own occupancy.
 *   GF_BATCH_QUEUE: one persistent kernel; workgroups take tiles from a
 *     queue ordered phase by phase and wait on per-image phase counters, so
 *     the phases of different images overlap.
 * tile_h: rows of the low-res coefficient tiles: 8, 16, 24, or 32 and 48
 * with GF_BATCH_PHASES.  A batch takes the tallest height up to tile_h
 * whose tiles fit in LDS at its largest r' (at most 24 under
 * GF_BATCH_QUEUE); 0 means up to 24.  Box-mean tiles take 48 rows under
 * GF_BATCH_PHASES where they fit, else the same height.
 */
typedef enum { GF_BATCH_PHASES = 0, GF_BATCH_QUEUE = 1 } gf_batch_schedule;

typedef struct {
    int32_t schedule; /* gf_batch_schedule */
    int32_t tile_h;
} gf_batch_cfg;

/* Schedule and tile height of the context's batched launches (gf_fast_batched,
 * gf_batch_create, gf_submit); NULL restores the default {GF_BATCH_PHASES, 0}.
 * GF_EINVAL for an unknown schedule or tile height. */
gf_status gf_ctx_set_batch_cfg(gf_ctx *ctx, const gf_batch_cfg *cfg);

/*
 * Bound of the waits in GF_BATCH_QUEUE launches made through ctx
 * (gf_fast_batched, gf_batch_create, gf_submit): a tile polls the counter of
 * its image's previous phase at most `polls` times (a poll sleeps about 50
 * ns) before it gives up, sets the batch's error word and skips its work, so
 * every launch ends even if a dependency never completes.  That image's q is
 * then incomplete: gf_fast_batched reports it in the workspace's error word,
 * gf_poll returns GF_EDEVICE for the requests of such a batch.  The default
 * (polls < 0) is about three seconds; 0 gives up at the first unfinished
 * dependency.  A prepared batch keeps the limit it was created with.
 * GF_EINVAL above 2^32 - 1.  The phase schedule has no waits.
 */
gf_status gf_ctx_set_wait_limit(gf_ctx *ctx, int64_t polls);

typedef struct {
    gf_batch_cfg cfg;
    double ms; /* mean time of one launch of the whole batch */
} gf_batch_tune_result;

/*
 * Autotuner for batches: times gf_fast_batched on this batch for every
 * tile height that fits (`reps` launches each, after one warm-up, HIP
 * events on `hip_stream`), of the phase schedule, or of the queue schedule
 * when the context's configuration is GF_BATCH_QUEUE, sets the fastest as
 * the context's batch configuration and writes it to *best.  Up to max_results timings go
 * to results (count in *n_results).  Arguments as gf_fast_batched; q holds
 * the batch's output when it returns.  Synchronises `hip_stream`.
 */
gf_status gf_tune_batched(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p, gf_image *q,
                          const gf_params *params, void *workspace, size_t workspace_bytes,
                          void *hip_stream, int32_t reps, gf_batch_cfg *best,
                          gf_batch_tune_result *results, int32_t max_results, int32_t *n_results);

/*
 * A prepared batch: the same work as gf_fast_batched, planned once so that
 * the launch itself can be captured into a HIP graph and replayed.
 *
 * gf_batch_create validates the n problems, lays out the tile queue and the
 * workspace, copies the descriptor table into the workspace and waits for
 * that copy on `hip_stream` (so it must not run under stream capture).  It
 * does not launch the filter.  `workspace` is device memory of at least
 * gf_batched_workspace_bytes(...) bytes owned by the caller (NULL is
 * refused: the batch keeps pointing at it).  The batch records the device
 * addresses in I, p, q and the workspace; those buffers must outlive it.
 * Returns GF_OK with *out set, or the errors of gf_fast_batched.
 *
 * gf_batch_launch enqueues the whole batch on `hip_stream`: a small kernel
 * that clears the queue's control words, then the persistent kernel (or,
 * for radii past the persistent kernel's tile limit, the per-image
 * kernels).  It copies nothing from the host, allocates nothing and never
 * synchronises, so it may be called under stream capture; every launch or
 * replay reads the current contents of I and p and rewrites q.  Launches of
 * one batch on different streams must not overlap (they share the
 * workspace).  ctx profiling does not apply to it.
 *
 * gf_batch_destroy frees the host-side plan (not the workspace, not any
 * graph holding its launch: destroy those first).
 */
typedef struct gf_batch gf_batch;

gf_status gf_batch_create(gf_ctx *ctx, int32_t n, const gf_image *I, const gf_image *p,
                          gf_image *q, const gf_params *params, void *workspace,
                          size_t workspace_bytes, void *hip_stream, gf_batch **out);
gf_status gf_batch_launch(const gf_batch *batch, void *hip_stream);
void gf_batch_destroy(gf_batch *batch);

/*
 * Asynchronous request: filter (I, p) into q like gf_fast.  The request is
 * admitted when the context's arena has room for its workspace, batched with
 * the other requests in flight, and run on the context's own streams.  A
 * request the batched kernels do not run (a colour guide, area subsampling,
 * a low-res radius above their limit) is admitted alone and runs the
 * per-image kernels; its q equals gf_fast's with the built-in tile shapes.
 * Returns GF_OK with *ticket set, GF_ENOMEM if it can never fit the arena,
 * GF_EBUSY if `max_inflight` requests are held, GF_EINVAL for bad arguments.
 * I, p, q must stay valid until gf_poll returns a terminal status.
 * Ordering: the context's streams do not wait for any stream of the caller.
 * The work that writes I and p must be complete when gf_submit is called
 * (for instance, the producing stream synchronised), and q may be read once
 * gf_poll has returned GF_OK (the library has then seen the batch's
 * completion event).
 */
gf_status gf_submit(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                    const gf_params *params, uint64_t *ticket);

/*
 * Status of a request: GF_PENDING while queued or running, GF_OK when q is
 * complete (the ticket is then retired), or the request's error.  Waits up
 * to `wait_ms` milliseconds for completion (0 = do not wait, negative = wait
 * without limit); GF_ETIMEDOUT if it is still pending after a positive wait.
 * `stats` (may be NULL) receives the request's timestamps on GF_OK.
 * Unknown or already retired tickets return GF_EINVAL.
 */
gf_status gf_poll(gf_ctx *ctx, uint64_t ticket, int32_t wait_ms, gf_req_stats *stats);

/*
 * Fusion of Algorithm 2 step 5 into steps 6-7.  With a gray guide at
 * s in {2, 4, 8} the box means of a and b can be formed inside the output
 * pass from a and b (two launches per call instead of three; mean_a and
 * mean_b never reach device memory) wherever the pass's LDS allows.  The
 * means are summed in the same order as by the separate box-mean pass with
 * the same tiles (gf_tiles.box_th), so q is the same, bit for bit, either
 * way; only the time differs.  GF_FUSE_AUTO (the default) fuses small
 * one-channel problems (c = 1, low-res maps of at most 65536 pixels), where
 * the launches are latency-bound; GF_FUSE_ON fuses wherever it applies;
 * GF_FUSE_OFF never.
 * The mode covers calls made through ctx (gf_plain, gf_fast,
 * gf_joint_upsample, gf_detail_enhance, gf_tune); calls without a context,
 * gf_fast_noalloc included, use GF_FUSE_AUTO.  GF_EINVAL for another mode.
 */
typedef enum { GF_FUSE_OFF = 0, GF_FUSE_AUTO = 1, GF_FUSE_ON = 2 } gf_fusion;
gf_status gf_ctx_set_fusion(gf_ctx *ctx, gf_fusion mode);

/*
 * Kernel timing for measurement.  While enabled on a context, every launch
 * made through it (gf_plain, gf_fast, gf_fast_batched) records a pair of HIP
 * events around each of its kernels on the caller's stream.
 * gf_ctx_profile_read waits for the recorded events, writes per-kernel
 * totals into out[0..GF_NKERNELS-1] (indexed by gf_kernel_id) and clears
 * them.  Enabling adds two event records per kernel; results are unchanged.
 */
typedef enum {
    GF_K_COEFF = 0,   /* subsample + window sums + a, b (Alg. 2 steps 1-4) */
    GF_K_BOX = 1,     /* box means of a, b (step 5) */
    GF_K_OUTPUT = 2,  /* bilinear upsample + q = mean_a*I + mean_b (steps 6-7) */
    GF_K_BATCHED = 3, /* the persistent kernel of gf_fast_batched */
    GF_K_AREA = 4,    /* area subsampling of I and p (GF_SUB_AREA only) */
    GF_NKERNELS = 5
} gf_kernel_id;

typedef struct {
    double total_ms;  /* summed event-to-event durations */
    int64_t launches;
} gf_kernel_time;

gf_status gf_ctx_profile(gf_ctx *ctx, int enable);
gf_status gf_ctx_profile_read(gf_ctx *ctx, gf_kernel_time *out);

/*
 * Tile shapes of the window-sum kernels (Algorithm 2 steps 2-5).  Both the
 * coefficient kernel and the box-mean kernel work on tiles of 64 low-res
 * columns by *_th rows (8, 16, 24, 32, 48 or 64) plus an r' halo staged in LDS.
 * Tall tiles amortise the halo; short ones need less LDS per workgroup.
 */
typedef struct {
    int32_t coeff_th;
    int32_t box_th;
} gf_tiles;

typedef struct {
    int32_t kernel;   /* GF_K_COEFF or GF_K_BOX */
    gf_tiles tiles;   /* the candidate (only that kernel's fields matter) */
    double ms;        /* mean duration of that kernel per call */
} gf_tune_result;

/*
 * Pin tile shapes on ctx for every call whose problem falls in the same
 * class as (h, w, c, params, dtype): same dtype, c, s, low-res radius r' and
 * size class (floor(log2(ceil(h/s) * ceil(w/s)))).  tiles == NULL removes
 * the pin (the built-in choice applies again).  GF_ENOTSUP if the shapes do
 * not fit in LDS for that radius.
 */
gf_status gf_ctx_set_tiles(gf_ctx *ctx, gf_dtype dtype, int32_t h, int32_t w, int32_t c,
                           const gf_params *params, const gf_tiles *tiles);

/*
 * Autotuner: times every candidate shape of the coefficient kernel and of
 * the box-mean kernel (where the box means are fused, of the fused output
 * pass, reported as GF_K_OUTPUT) on this problem (HIP events on `hip_stream`, `reps`
 * launches each after one warm-up), keeps the fastest of each for the
 * problem's class on ctx (as gf_ctx_set_tiles would) and returns it in
 * *best (may be NULL).  Synchronises the stream; q's contents are
 * overwritten with a valid result.  results (may be NULL) receive up to
 * max_results timings, *n_results their count.  Same arguments and
 * workspace as gf_fast.
 */
gf_status gf_tune(gf_ctx *ctx, const gf_image *I, const gf_image *p, gf_image *q,
                  const gf_params *params, void *workspace, size_t workspace_bytes,
                  void *hip_stream, int32_t reps, gf_tiles *best, gf_tune_result *results,
                  int32_t max_results, int32_t *n_results);

/* Write the context's tuned shapes to a JSON file / read them back (entries
 * of the file replace those of the same class). */
gf_status gf_ctx_save_tuning(gf_ctx *ctx, const char *path);
gf_status gf_ctx_load_tuning(gf_ctx *ctx, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */
