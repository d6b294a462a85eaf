/*
 * FP64 CPU oracle for the guided filter and the Fast Guided Filter
 * (He & Sun, "Fast Guided Filter", arXiv 1505.00996).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  It is used by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg, and by nothing else.
 * It shares no code, header, table or constant with the HIP path.
 *
 * Everything is double precision, single threaded, with explicit loops.
 * Images are dense row-major arrays: pixel (y, x) of an h-by-w image is at
 * index y*w + x; channel k of a c-channel image starts at k*h*w.
 *
 * Conventions where the paper is silent (each is listed with its reason in
 * the design notes of the repository):
 *   - a window of radius r is the (2r+1)x(2r+1) square centred on a pixel
 *     (Sec. 2, below Eq. 1);
 *   - the mean filter f_mean averages over the part of the window that lies
 *     inside the image (clip-normalised border), which makes the average of
 *     the a_k over all windows containing pixel i (Eq. 4) a box mean;
 *   - the variance is the population variance, corr_I - mean_I^2, exactly as
 *     Algorithm 1 step 2 writes it; it is not clamped;
 *   - the low-resolution radius is r/s rounded half up, at least 1 when r>0;
 *   - low-resolution size is ceil(h/s) x ceil(w/s); geometry uses exactly s;
 *   - nearest-neighbour subsampling takes full-res index s*y + floor(s/2),
 *     clamped to the image; bilinear subsampling samples the low-res pixel
 *     centre s*y + (s-1)/2 with two clamped taps (no antialias prefilter);
 *   - bilinear upsampling uses half-pixel centres, u = (y+0.5)/s - 0.5, with
 *     taps clamped to the low-res map;
 *   - a multi-channel p is filtered channel by channel with the same gray I;
 *   - optional conventions of other libraries: a padded border, where the
 *     image is extended past its edges (replicating the edge pixel, or
 *     mirroring about it without repeating it: "reflect-101") and every
 *     window mean divides by (2r+1)^2; and area subsampling, the mean of the
 *     s x s block of full-res pixels [s*y, s*y+s) x [s*x, s*x+s) restricted
 *     to the image.
 *
 * Parity status: every function here is pinned by the CPU tests (brute-force
 * window loops, scipy/torch special cases, a least-squares solve of the
 * windowed ridge regression, and closed-form invariants of Eqs. 1-4; joint
 * upsampling against its assembly from library routines and against the fast
 * filter of a subsampled input; detail enhancement at its gain end points;
 * the padded borders against numpy's edge and reflect padding and scipy's
 * uniform filter, area subsampling against torch's average pooling; colour
 * guidance against a least-squares solve of its windowed ridge regression,
 * a library assembly, and the gray filter for a guide of three equal planes).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NEAREST 0
#define ORACLE_BILINEAR 1
#define ORACLE_AREA 2

#define ORACLE_CLIP 0
#define ORACLE_REPLICATE 1
#define ORACLE_REFLECT101 2

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static int iclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Low-resolution radius r' = r/s (Algorithm 2, step 1), rounded half up with
 * integer arithmetic; at least 1 when r > 0 so a window never collapses. */
int oracle_lowres_radius(int r, int s)
{
    if (r <= 0) return 0;
    int rl = (2 * r + s) / (2 * s);
    return rl < 1 ? 1 : rl;
}

/* Low-resolution extent of an n-pixel axis subsampled by s: ceil(n/s). */
int oracle_lowres_size(int n, int s) { return (n + s - 1) / s; }

/*
 * f_mean(x, r) of Algorithm 1: for every pixel, the mean of x over the
 * (2r+1)x(2r+1) window centred on it, restricted to the image and divided by
 * the number of in-image pixels of that window.  The double sum over the
 * window is taken as a sum over rows of sums along each row; the window
 * count is the product of the clipped row and column extents.
 */
int oracle_box_mean(const double *x, int h, int w, int r, double *out)
{
    if (h <= 0 || w <= 0 || r < 0) return -1;
    double *rowsum = (double *)malloc(sizeof(double) * (size_t)h * (size_t)w);
    double *acc = (double *)malloc(sizeof(double) * (size_t)w);
    if (!rowsum || !acc) { free(rowsum); free(acc); return -2; }

    for (int y = 0; y < h; ++y) {
        const double *src = x + (size_t)y * w;
        double *dst = rowsum + (size_t)y * w;
        for (int xx = 0; xx < w; ++xx) {
            double s = 0.0;
            for (int k = imax(0, xx - r); k <= imin(w - 1, xx + r); ++k) s += src[k];
            dst[xx] = s;
        }
    }
    for (int y = 0; y < h; ++y) {
        int y0 = imax(0, y - r), y1 = imin(h - 1, y + r);
        for (int xx = 0; xx < w; ++xx) acc[xx] = 0.0;
        /* rows are added in ascending order, the same order as a plain
         * per-pixel loop over the window rows */
        for (int k = y0; k <= y1; ++k) {
            const double *src = rowsum + (size_t)k * w;
            for (int xx = 0; xx < w; ++xx) acc[xx] += src[xx];
        }
        double *dst = out + (size_t)y * w;
        for (int xx = 0; xx < w; ++xx) {
            int x0 = imax(0, xx - r), x1 = imin(w - 1, xx + r);
            double count = (double)(y1 - y0 + 1) * (double)(x1 - x0 + 1);
            dst[xx] = acc[xx] / count;
        }
    }
    free(rowsum);
    free(acc);
    return 0;
}

/*
 * Position i of an n-pixel axis extended past its ends, as an index into the
 * axis.  Replicate repeats the end pixel.  Reflect-101 mirrors the axis about
 * its first and last pixels without repeating them (... 2 1 | 0 1 2 ... n-1 |
 * n-2 n-3 ...), as many times as a window wider than the axis needs; a
 * one-pixel axis is that pixel everywhere.
 */
static int border_index(int i, int n, int border)
{
    if (border == ORACLE_REPLICATE) return iclamp(i, 0, n - 1);
    if (n == 1) return 0;
    while (i < 0 || i > n - 1) {
        if (i < 0) i = -i;
        if (i > n - 1) i = 2 * (n - 1) - i;
    }
    return i;
}

/*
 * f_mean with a padded border: every pixel's (2r+1)x(2r+1) window reads the
 * image extended past its edges (border_index), so every window holds
 * (2r+1)^2 samples and the mean divides by that.  Row sums first, then the
 * sum of 2r+1 row sums, both in window order.
 */
static int box_mean_padded(const double *x, int h, int w, int r, int border, double *out)
{
    double *rowsum = (double *)malloc(sizeof(double) * (size_t)h * (size_t)w);
    if (!rowsum) return -2;
    for (int y = 0; y < h; ++y) {
        for (int xx = 0; xx < w; ++xx) {
            double acc = 0.0;
            for (int k = -r; k <= r; ++k) acc += x[(size_t)y * w + border_index(xx + k, w, border)];
            rowsum[(size_t)y * w + xx] = acc;
        }
    }
    const double count = (double)(2 * r + 1) * (double)(2 * r + 1);
    for (int y = 0; y < h; ++y) {
        for (int xx = 0; xx < w; ++xx) {
            double acc = 0.0;
            for (int k = -r; k <= r; ++k) acc += rowsum[(size_t)border_index(y + k, h, border) * w + xx];
            out[(size_t)y * w + xx] = acc / count;
        }
    }
    free(rowsum);
    return 0;
}

/* f_mean under the given border convention (clip-normalised, replicate or
 * reflect-101). */
int oracle_box_mean_border(const double *x, int h, int w, int r, int border, double *out)
{
    if (border == ORACLE_CLIP) return oracle_box_mean(x, h, w, r, out);
    if (h <= 0 || w <= 0 || r < 0) return -1;
    if (border != ORACLE_REPLICATE && border != ORACLE_REFLECT101) return -1;
    return box_mean_padded(x, h, w, r, border, out);
}

/*
 * f_subsample(x, s) of Algorithm 2, step 1 (the paper allows nearest-neighbour
 * or bilinear).  Output is ceil(h/s) x ceil(w/s).
 *   nearest : x(min(s*y + s/2, h-1), min(s*x + s/2, w-1)).
 *   bilinear: point sample at the low-res pixel centre u = s*y + (s-1)/2
 *             (half-pixel convention), taps floor(u), floor(u)+1 clamped.
 */
static void axis_sample(int j, int s, int n, int mode, int *t0, int *t1, double *wt)
{
    if (mode == ORACLE_NEAREST) {
        *t0 = imin(s * j + s / 2, n - 1);
        *t1 = *t0;
        *wt = 0.0;
        return;
    }
    double u = (double)s * j + 0.5 * (double)(s - 1);
    double f = floor(u);
    *wt = u - f;
    *t0 = iclamp((int)f, 0, n - 1);
    *t1 = iclamp((int)f + 1, 0, n - 1);
}

/*
 * Area subsampling: low-res pixel (y, x) is the mean of the full-res pixels
 * of the block [s*y, s*y+s) x [s*x, s*x+s) that lie inside the image (the
 * last block of an axis whose length is not a multiple of s is shorter).
 */
static void area_subsample(const double *x, int h, int w, int s, double *out)
{
    int hl = oracle_lowres_size(h, s), wl = oracle_lowres_size(w, s);
    for (int y = 0; y < hl; ++y) {
        int y0 = s * y, y1 = imin(h, s * y + s);
        for (int xx = 0; xx < wl; ++xx) {
            int x0 = s * xx, x1 = imin(w, s * xx + s);
            double acc = 0.0;
            for (int i = y0; i < y1; ++i)
                for (int j = x0; j < x1; ++j) acc += x[(size_t)i * w + j];
            out[(size_t)y * wl + xx] = acc / ((double)(y1 - y0) * (double)(x1 - x0));
        }
    }
}

int oracle_subsample(const double *x, int h, int w, int s, int mode, double *out)
{
    if (h <= 0 || w <= 0 || s < 1) return -1;
    if (mode == ORACLE_AREA) {
        area_subsample(x, h, w, s, out);
        return 0;
    }
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR) return -1;
    int hl = oracle_lowres_size(h, s), wl = oracle_lowres_size(w, s);
    for (int y = 0; y < hl; ++y) {
        int ya, yb;
        double wy;
        axis_sample(y, s, h, mode, &ya, &yb, &wy);
        for (int xx = 0; xx < wl; ++xx) {
            int xa, xb;
            double wx;
            axis_sample(xx, s, w, mode, &xa, &xb, &wx);
            double v00 = x[(size_t)ya * w + xa], v01 = x[(size_t)ya * w + xb];
            double v10 = x[(size_t)yb * w + xa], v11 = x[(size_t)yb * w + xb];
            out[(size_t)y * wl + xx] =
                (1.0 - wy) * ((1.0 - wx) * v00 + wx * v01) + wy * ((1.0 - wx) * v10 + wx * v11);
        }
    }
    return 0;
}

/*
 * f_upsample(x, s) of Algorithm 2, step 6: bilinear interpolation of an
 * hl x wl map back to h x w.  Full-res pixel y sits at low-res coordinate
 * u = (y + 0.5)/s - 0.5; the taps floor(u) and floor(u)+1 are clamped to the
 * low-res map, with weight u - floor(u) on the second.
 */
int oracle_upsample(const double *lo, int hl, int wl, int s, int h, int w, double *out)
{
    if (hl <= 0 || wl <= 0 || h <= 0 || w <= 0 || s < 1) return -1;
    for (int y = 0; y < h; ++y) {
        double u = ((double)y + 0.5) / (double)s - 0.5;
        double fu = floor(u);
        double wy = u - fu;
        int ya = iclamp((int)fu, 0, hl - 1), yb = iclamp((int)fu + 1, 0, hl - 1);
        for (int xx = 0; xx < w; ++xx) {
            double v = ((double)xx + 0.5) / (double)s - 0.5;
            double fv = floor(v);
            double wx = v - fv;
            int xa = iclamp((int)fv, 0, wl - 1), xb = iclamp((int)fv + 1, 0, wl - 1);
            double v00 = lo[(size_t)ya * wl + xa], v01 = lo[(size_t)ya * wl + xb];
            double v10 = lo[(size_t)yb * wl + xa], v11 = lo[(size_t)yb * wl + xb];
            out[(size_t)y * w + xx] =
                (1.0 - wy) * ((1.0 - wx) * v00 + wx * v01) + wy * ((1.0 - wx) * v10 + wx * v11);
        }
    }
    return 0;
}

/*
 * Algorithm 1, steps 1-3, for one channel of p: the per-window linear
 * coefficients of Eqs. 2-3,
 *   a = (mean(I.*p) - mean(I) mean(p)) / (var(I) + eps),  b = mean(p) - a mean(I),
 * with every mean a box mean of radius r under the border convention.
 */
static int coefficients(const double *I, const double *p, int h, int w, int r, double eps, int border,
                        double *a, double *b)
{
    size_t n = (size_t)h * (size_t)w;
    double *mean_I = (double *)malloc(sizeof(double) * n);
    double *mean_p = (double *)malloc(sizeof(double) * n);
    double *corr_I = (double *)malloc(sizeof(double) * n);
    double *corr_Ip = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!mean_I || !mean_p || !corr_I || !corr_Ip || !tmp) { rc = -2; goto done; }

    /* step 1: four mean filters; the products are formed pixel by pixel first */
    if ((rc = oracle_box_mean_border(I, h, w, r, border, mean_I))) goto done;
    if ((rc = oracle_box_mean_border(p, h, w, r, border, mean_p))) goto done;
    for (size_t i = 0; i < n; ++i) tmp[i] = I[i] * I[i];
    if ((rc = oracle_box_mean_border(tmp, h, w, r, border, corr_I))) goto done;
    for (size_t i = 0; i < n; ++i) tmp[i] = I[i] * p[i];
    if ((rc = oracle_box_mean_border(tmp, h, w, r, border, corr_Ip))) goto done;

    /* steps 2-3: variance, covariance, then the closed forms of Eqs. 2-3 */
    for (size_t i = 0; i < n; ++i) {
        double var_I = corr_I[i] - mean_I[i] * mean_I[i];
        double cov_Ip = corr_Ip[i] - mean_I[i] * mean_p[i];
        a[i] = cov_Ip / (var_I + eps);
        b[i] = mean_p[i] - a[i] * mean_I[i];
    }
done:
    free(mean_I); free(mean_p); free(corr_I); free(corr_Ip); free(tmp);
    return rc;
}

int oracle_coefficients(const double *I, const double *p, int h, int w, int r, double eps,
                        double *a, double *b)
{
    return coefficients(I, p, h, w, r, eps, ORACLE_CLIP, a, b);
}

/*
 * Algorithm 1 (the guided filter) for a c-channel p with gray guide I.
 * Per channel: a, b from Eqs. 2-3 (steps 1-3), their box means (step 4) and
 * q = mean_a .* I + mean_b (step 5, Eq. 4).
 * Optional outputs (may be NULL), c*h*w each: a, b, mean_a, mean_b.
 * Every mean uses the border convention `border` (ORACLE_CLIP: clip-normalised).
 */
int oracle_guided_filter_ex(const double *I, const double *p, int c, int h, int w, int r,
                            double eps, int border, double *q, double *a_out, double *b_out,
                            double *mean_a_out, double *mean_b_out)
{
    if (h <= 0 || w <= 0 || c <= 0 || r < 0 || !(eps > 0.0)) return -1;
    size_t n = (size_t)h * (size_t)w;
    double *a = (double *)malloc(sizeof(double) * n);
    double *b = (double *)malloc(sizeof(double) * n);
    double *ma = (double *)malloc(sizeof(double) * n);
    double *mb = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!a || !b || !ma || !mb) { rc = -2; goto done; }
    for (int k = 0; k < c; ++k) {
        const double *pk = p + (size_t)k * n;
        double *qk = q + (size_t)k * n;
        if ((rc = coefficients(I, pk, h, w, r, eps, border, a, b))) goto done;
        if ((rc = oracle_box_mean_border(a, h, w, r, border, ma))) goto done;
        if ((rc = oracle_box_mean_border(b, h, w, r, border, mb))) goto done;
        for (size_t i = 0; i < n; ++i) qk[i] = ma[i] * I[i] + mb[i];
        if (a_out) memcpy(a_out + (size_t)k * n, a, sizeof(double) * n);
        if (b_out) memcpy(b_out + (size_t)k * n, b, sizeof(double) * n);
        if (mean_a_out) memcpy(mean_a_out + (size_t)k * n, ma, sizeof(double) * n);
        if (mean_b_out) memcpy(mean_b_out + (size_t)k * n, mb, sizeof(double) * n);
    }
done:
    free(a); free(b); free(ma); free(mb);
    return rc;
}

int oracle_guided_filter(const double *I, const double *p, int c, int h, int w, int r,
                         double eps, double *q, double *a_out, double *b_out,
                         double *mean_a_out, double *mean_b_out)
{
    return oracle_guided_filter_ex(I, p, c, h, w, r, eps, ORACLE_CLIP, q, a_out, b_out, mean_a_out,
                                   mean_b_out);
}

/*
 * Algorithm 2 (the Fast Guided Filter) for a c-channel p with gray guide I.
 *   step 1: I' = f_subsample(I, s), p' = f_subsample(p, s), r' = r/s;
 *   steps 2-5: Algorithm 1 steps 1-4 on I', p' at radius r' -> mean_a, mean_b;
 *   step 6: mean_a, mean_b bilinearly upsampled to h x w;
 *   step 7: q = mean_a .* I + mean_b against the full-resolution I.
 * Optional low-resolution outputs (may be NULL), c*hl*wl each: a, b,
 * mean_a, mean_b before upsampling.  `mode` is the subsampling (nearest,
 * bilinear or area); every low-res mean uses the border convention `border`.
 */
int oracle_fast_guided_filter_ex(const double *I, const double *p, int c, int h, int w, int r,
                                 int s, double eps, int mode, int border, double *q, double *a_lo,
                                 double *b_lo, double *mean_a_lo, double *mean_b_lo)
{
    if (h <= 0 || w <= 0 || c <= 0 || r < 0 || s < 1 || !(eps > 0.0)) return -1;
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR && mode != ORACLE_AREA) return -1;
    int hl = oracle_lowres_size(h, s), wl = oracle_lowres_size(w, s);
    int rl = oracle_lowres_radius(r, s);
    size_t n = (size_t)h * (size_t)w, nl = (size_t)hl * (size_t)wl;
    double *Il = (double *)malloc(sizeof(double) * nl);
    double *pl = (double *)malloc(sizeof(double) * nl);
    double *a = (double *)malloc(sizeof(double) * nl);
    double *b = (double *)malloc(sizeof(double) * nl);
    double *ma = (double *)malloc(sizeof(double) * nl);
    double *mb = (double *)malloc(sizeof(double) * nl);
    double *ua = (double *)malloc(sizeof(double) * n);
    double *ub = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!Il || !pl || !a || !b || !ma || !mb || !ua || !ub) { rc = -2; goto done; }

    if ((rc = oracle_subsample(I, h, w, s, mode, Il))) goto done;
    for (int k = 0; k < c; ++k) {
        const double *pk = p + (size_t)k * n;
        double *qk = q + (size_t)k * n;
        if ((rc = oracle_subsample(pk, h, w, s, mode, pl))) goto done;
        if ((rc = coefficients(Il, pl, hl, wl, rl, eps, border, a, b))) goto done;
        if ((rc = oracle_box_mean_border(a, hl, wl, rl, border, ma))) goto done;
        if ((rc = oracle_box_mean_border(b, hl, wl, rl, border, mb))) goto done;
        if ((rc = oracle_upsample(ma, hl, wl, s, h, w, ua))) goto done;
        if ((rc = oracle_upsample(mb, hl, wl, s, h, w, ub))) goto done;
        for (size_t i = 0; i < n; ++i) qk[i] = ua[i] * I[i] + ub[i];
        if (a_lo) memcpy(a_lo + (size_t)k * nl, a, sizeof(double) * nl);
        if (b_lo) memcpy(b_lo + (size_t)k * nl, b, sizeof(double) * nl);
        if (mean_a_lo) memcpy(mean_a_lo + (size_t)k * nl, ma, sizeof(double) * nl);
        if (mean_b_lo) memcpy(mean_b_lo + (size_t)k * nl, mb, sizeof(double) * nl);
    }
done:
    free(Il); free(pl); free(a); free(b); free(ma); free(mb); free(ua); free(ub);
    return rc;
}

int oracle_fast_guided_filter(const double *I, const double *p, int c, int h, int w, int r,
                              int s, double eps, int mode, double *q, double *a_lo,
                              double *b_lo, double *mean_a_lo, double *mean_b_lo)
{
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR) return -1;
    return oracle_fast_guided_filter_ex(I, p, c, h, w, r, s, eps, mode, ORACLE_CLIP, q, a_lo, b_lo,
                                        mean_a_lo, mean_b_lo);
}

/*
 * Joint upsampling (the use of the subsampling the paper's introduction
 * mentions): the input is given at low resolution, p_lo with c channels of
 * ceil(h/s) x ceil(w/s), and only the full-resolution guide is subsampled
 * (Algorithm 2 step 1 for I alone).  Steps 2-7 of Algorithm 2 then run
 * unchanged with p' = p_lo: coefficients at r' = r/s, their box means,
 * bilinear upsampling, q = mean_a .* I + mean_b on the full-resolution I.
 * Subsampling `mode` and border convention `border` as in the fast filter.
 */
int oracle_joint_upsample_ex(const double *I, const double *p_lo, int c, int h, int w, int r, int s,
                             double eps, int mode, int border, double *q)
{
    if (h <= 0 || w <= 0 || c <= 0 || r < 0 || s < 1 || !(eps > 0.0)) return -1;
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR && mode != ORACLE_AREA) return -1;
    int hs = oracle_lowres_size(h, s), ws = oracle_lowres_size(w, s);
    int rs = oracle_lowres_radius(r, s);
    size_t n = (size_t)h * (size_t)w, ns = (size_t)hs * (size_t)ws;
    double *Is = (double *)malloc(sizeof(double) * ns);
    double *ak = (double *)malloc(sizeof(double) * ns);
    double *bk = (double *)malloc(sizeof(double) * ns);
    double *mak = (double *)malloc(sizeof(double) * ns);
    double *mbk = (double *)malloc(sizeof(double) * ns);
    double *uak = (double *)malloc(sizeof(double) * n);
    double *ubk = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!Is || !ak || !bk || !mak || !mbk || !uak || !ubk) { rc = -2; goto done; }

    if ((rc = oracle_subsample(I, h, w, s, mode, Is))) goto done;   /* the guide only */
    for (int k = 0; k < c; ++k) {
        const double *pc = p_lo + (size_t)k * ns;                   /* p' is given */
        double *qc = q + (size_t)k * n;
        if ((rc = coefficients(Is, pc, hs, ws, rs, eps, border, ak, bk))) goto done;
        if ((rc = oracle_box_mean_border(ak, hs, ws, rs, border, mak))) goto done;
        if ((rc = oracle_box_mean_border(bk, hs, ws, rs, border, mbk))) goto done;
        if ((rc = oracle_upsample(mak, hs, ws, s, h, w, uak))) goto done;
        if ((rc = oracle_upsample(mbk, hs, ws, s, h, w, ubk))) goto done;
        for (size_t i = 0; i < n; ++i) qc[i] = uak[i] * I[i] + ubk[i];
    }
done:
    free(Is); free(ak); free(bk); free(mak); free(mbk); free(uak); free(ubk);
    return rc;
}

int oracle_joint_upsample(const double *I, const double *p_lo, int c, int h, int w, int r, int s,
                          double eps, int mode, double *q)
{
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR) return -1;
    return oracle_joint_upsample_ex(I, p_lo, c, h, w, r, s, eps, mode, ORACLE_CLIP, q);
}

/*
 * Colour guidance (a three-channel guide I = (I0, I1, I2), planes of h*w).
 * The paper names the number of channels as a cost factor and takes the
 * colour form of the guided filter from its earlier definition: in every
 * window the linear model is q = a^T I + b with a a 3-vector, fitted by
 *   min  sum_{i in w_k} (a^T I_i + b - p_i)^2 + eps |a|^2
 * (the same ridge regression as the gray Eqs. 1-3, one eps|a|^2 per pixel),
 * whose solution is
 *   a_k = (Sigma_k + eps U)^-1 (mean(I p) - mean(I) mean(p)),  b_k = mean(p) - a_k^T mean(I),
 * with Sigma_k the 3x3 population covariance of I in the window and U the
 * identity; q_i = mean_a(i)^T I_i + mean_b(i) with the box means of Eq. 4.
 */

/* x = M^-1 y for a 3x3 matrix M (row-major), by its adjugate and determinant. */
static void solve3(const double M[9], const double y[3], double x[3])
{
    double adj[9];
    adj[0] = M[4] * M[8] - M[5] * M[7];
    adj[1] = M[2] * M[7] - M[1] * M[8];
    adj[2] = M[1] * M[5] - M[2] * M[4];
    adj[3] = M[5] * M[6] - M[3] * M[8];
    adj[4] = M[0] * M[8] - M[2] * M[6];
    adj[5] = M[2] * M[3] - M[0] * M[5];
    adj[6] = M[3] * M[7] - M[4] * M[6];
    adj[7] = M[1] * M[6] - M[0] * M[7];
    adj[8] = M[0] * M[4] - M[1] * M[3];
    double det = M[0] * adj[0] + M[1] * adj[3] + M[2] * adj[6];
    for (int r = 0; r < 3; ++r)
        x[r] = (adj[3 * r] * y[0] + adj[3 * r + 1] * y[1] + adj[3 * r + 2] * y[2]) / det;
}

/*
 * Coefficients of the colour model for one channel of p: a (3 planes a0, a1,
 * a2 of n = h*w) and b, every mean a box mean of radius r under `border`.
 */
static int coefficients_color(const double *I, const double *p, int h, int w, int r, double eps, int border,
                              double *a, double *b)
{
    size_t n = (size_t)h * (size_t)w;
    double *mI = (double *)malloc(sizeof(double) * 3 * n);    /* mean of I_j */
    double *cII = (double *)malloc(sizeof(double) * 9 * n);   /* mean of I_j I_k */
    double *cIp = (double *)malloc(sizeof(double) * 3 * n);   /* mean of I_j p */
    double *mp = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!mI || !cII || !cIp || !mp || !tmp) { rc = -2; goto done; }
    if ((rc = oracle_box_mean_border(p, h, w, r, border, mp))) goto done;
    for (int j = 0; j < 3; ++j) {
        const double *Ij = I + (size_t)j * n;
        if ((rc = oracle_box_mean_border(Ij, h, w, r, border, mI + (size_t)j * n))) goto done;
        for (size_t i = 0; i < n; ++i) tmp[i] = Ij[i] * p[i];
        if ((rc = oracle_box_mean_border(tmp, h, w, r, border, cIp + (size_t)j * n))) goto done;
        for (int k = 0; k < 3; ++k) {
            const double *Ik = I + (size_t)k * n;
            for (size_t i = 0; i < n; ++i) tmp[i] = Ij[i] * Ik[i];
            if ((rc = oracle_box_mean_border(tmp, h, w, r, border, cII + (size_t)(3 * j + k) * n))) goto done;
        }
    }
    for (size_t i = 0; i < n; ++i) {
        double M[9], cov[3], x[3];
        for (int j = 0; j < 3; ++j) {
            for (int k = 0; k < 3; ++k)
                M[3 * j + k] = cII[(size_t)(3 * j + k) * n + i] - mI[(size_t)j * n + i] * mI[(size_t)k * n + i];
            M[3 * j + j] += eps;
            cov[j] = cIp[(size_t)j * n + i] - mI[(size_t)j * n + i] * mp[i];
        }
        solve3(M, cov, x);
        double bi = mp[i];
        for (int j = 0; j < 3; ++j) {
            a[(size_t)j * n + i] = x[j];
            bi -= x[j] * mI[(size_t)j * n + i];
        }
        b[i] = bi;
    }
done:
    free(mI); free(cII); free(cIp); free(mp); free(tmp);
    return rc;
}

/*
 * The fast guided filter with a colour guide: I has 3 planes (h x w), p has c.
 * Step 1 subsamples every plane of I and p (s = 1: the guided filter itself);
 * a (3 per channel) and b at r' = r/s; their box means; bilinear upsampling;
 * q = mean_a0 I0 + mean_a1 I1 + mean_a2 I2 + mean_b on the full-res guide.
 * Optional outputs (may be NULL), low resolution: a_lo (c*3*hl*wl, channel k's
 * three planes at 3k..3k+2), b_lo (c*hl*wl).
 */
int oracle_fast_guided_filter_color(const double *I, const double *p, int c, int h, int w, int r, int s,
                                    double eps, int mode, int border, double *q, double *a_lo, double *b_lo)
{
    if (h <= 0 || w <= 0 || c <= 0 || r < 0 || s < 1 || !(eps > 0.0)) return -1;
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR && mode != ORACLE_AREA) return -1;
    int hl = oracle_lowres_size(h, s), wl = oracle_lowres_size(w, s);
    int rl = oracle_lowres_radius(r, s);
    size_t n = (size_t)h * (size_t)w, nl = (size_t)hl * (size_t)wl;
    double *Il = (double *)malloc(sizeof(double) * 3 * nl);
    double *pl = (double *)malloc(sizeof(double) * nl);
    double *ca = (double *)malloc(sizeof(double) * 3 * nl);
    double *cb = (double *)malloc(sizeof(double) * nl);
    double *mean_lo = (double *)malloc(sizeof(double) * nl);
    double *up = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!Il || !pl || !ca || !cb || !mean_lo || !up) { rc = -2; goto done; }
    for (int j = 0; j < 3; ++j)
        if ((rc = oracle_subsample(I + (size_t)j * n, h, w, s, mode, Il + (size_t)j * nl))) goto done;
    for (int k = 0; k < c; ++k) {
        double *qk = q + (size_t)k * n;
        if ((rc = oracle_subsample(p + (size_t)k * n, h, w, s, mode, pl))) goto done;
        if ((rc = coefficients_color(Il, pl, hl, wl, rl, eps, border, ca, cb))) goto done;
        if (a_lo) memcpy(a_lo + (size_t)3 * k * nl, ca, sizeof(double) * 3 * nl);
        if (b_lo) memcpy(b_lo + (size_t)k * nl, cb, sizeof(double) * nl);
        /* q = sum_j up(mean(a_j)) I_j + up(mean(b)), terms added in that order */
        for (size_t i = 0; i < n; ++i) qk[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
            if ((rc = oracle_box_mean_border(ca + (size_t)j * nl, hl, wl, rl, border, mean_lo))) goto done;
            if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;
            const double *Ij = I + (size_t)j * n;
            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * Ij[i];
        }
        if ((rc = oracle_box_mean_border(cb, hl, wl, rl, border, mean_lo))) goto done;
        if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;
        for (size_t i = 0; i < n; ++i) qk[i] += up[i];
    }
done:
    free(Il); free(pl); free(ca); free(cb); free(mean_lo); free(up);
    return rc;
}

/*
 * Joint upsampling with a colour guide: p_lo (c planes of ceil(h/s) x
 * ceil(w/s)) is given at low resolution, only the three guide planes are
 * subsampled, and the colour filter's remaining steps run as in
 * oracle_fast_guided_filter_color.
 */
int oracle_joint_upsample_color(const double *I, const double *p_lo, int c, int h, int w, int r, int s,
                                double eps, int mode, int border, double *q)
{
    if (h <= 0 || w <= 0 || c <= 0 || r < 0 || s < 1 || !(eps > 0.0)) return -1;
    if (mode != ORACLE_NEAREST && mode != ORACLE_BILINEAR && mode != ORACLE_AREA) return -1;
    int hl = oracle_lowres_size(h, s), wl = oracle_lowres_size(w, s);
    int rl = oracle_lowres_radius(r, s);
    size_t n = (size_t)h * (size_t)w, nl = (size_t)hl * (size_t)wl;
    double *Il = (double *)malloc(sizeof(double) * 3 * nl);
    double *ca = (double *)malloc(sizeof(double) * 3 * nl);
    double *cb = (double *)malloc(sizeof(double) * nl);
    double *mean_lo = (double *)malloc(sizeof(double) * nl);
    double *up = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!Il || !ca || !cb || !mean_lo || !up) { rc = -2; goto done; }
    for (int j = 0; j < 3; ++j)
        if ((rc = oracle_subsample(I + (size_t)j * n, h, w, s, mode, Il + (size_t)j * nl))) goto done;
    for (int k = 0; k < c; ++k) {
        double *qk = q + (size_t)k * n;
        if ((rc = coefficients_color(Il, p_lo + (size_t)k * nl, hl, wl, rl, eps, border, ca, cb))) goto done;
        for (size_t i = 0; i < n; ++i) qk[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
            if ((rc = oracle_box_mean_border(ca + (size_t)j * nl, hl, wl, rl, border, mean_lo))) goto done;
            if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;
            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * I[(size_t)j * n + i];
        }
        if ((rc = oracle_box_mean_border(cb, hl, wl, rl, border, mean_lo))) goto done;
        if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;
        for (size_t i = 0; i < n; ++i) qk[i] += up[i];
    }
done:
    free(Il); free(ca); free(cb); free(mean_lo); free(up);
    return rc;
}

/*
 * Detail enhancement, the paper's first application: the filtered image q is
 * the base layer, p - q the detail layer, and the enhanced image carries the
 * detail `gain` times over (its example shows x5 detail):
 *   e = q + gain * (p - q).
 */
int oracle_detail_enhance(const double *p, const double *q, size_t n, double gain, double *e)
{
    if (!p || !q || !e) return -1;
    for (size_t i = 0; i < n; ++i) e[i] = q[i] + gain * (p[i] - q[i]);
    return 0;
}
