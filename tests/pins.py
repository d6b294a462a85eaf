"""Pins for the FP64 oracle: checks against things other than the oracle itself.

Each ``pin_*`` takes a loaded oracle (``oracle.oracle.Oracle``) and raises
AssertionError when the oracle disagrees with:
  * brute-force window loops on tiny images (dyadic values make the sums exact),
  * library routines for the special cases they cover (scipy's uniform filter,
    torch's interpolate, numpy's least-squares solver),
  * closed-form consequences of the local linear model (Eqs. 1-4).

The same pins run against the real oracle (tests/test_oracle.py) and against
deliberately broken copies of it (tests/test_oracle_mutants.py), which shows
that a plausible slip anywhere in the oracle fails at least one of them.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage as ndi
import torch
import torch.nn.functional as F


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dyadic(g, shape):
    return g.integers(0, 257, size=shape).astype(np.float64) / 256.0


def _close(got, exp, tol, what):
    got, exp = np.asarray(got), np.asarray(exp)
    assert got.shape == exp.shape, f"{what}: shape {got.shape} != {exp.shape}"
    err = float(np.max(np.abs(got - exp))) if got.size else 0.0
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    assert err <= tol, f"{what}: max abs err {err:.3e} > {tol:.1e}"


def _window(n, i, r):
    return max(0, i - r), min(n - 1, i + r)


def scipy_box(x, r):
    """Clip-normalised box mean from scipy's zero-padded uniform filter."""
    x = np.asarray(x, dtype=np.float64)
    size = 2 * r + 1
    num = ndi.uniform_filter(x, size=size, mode="constant", cval=0.0)
    den = ndi.uniform_filter(np.ones_like(x), size=size, mode="constant", cval=0.0)
    return num / den


def torch_nearest_sub(x, s):
    """torch 'nearest-exact' downscale by s (sizes divisible by s)."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))[None, None]
    h, w = x.shape
    return F.interpolate(t, size=(h // s, w // s), mode="nearest-exact")[0, 0].numpy()


def torch_bilinear_sub(x, s):
    """torch bilinear downscale by s, half-pixel centres, no antialias (s | h, w)."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))[None, None]
    h, w = x.shape
    return F.interpolate(t, size=(h // s, w // s), mode="bilinear", align_corners=False,
                         antialias=False)[0, 0].numpy()


def torch_upsample(lo, s, h, w):
    """torch bilinear upscale by exactly s (half-pixel centres), cropped to h x w."""
    t = torch.from_numpy(np.ascontiguousarray(lo, dtype=np.float64))[None, None]
    up = F.interpolate(t, scale_factor=float(s), mode="bilinear", align_corners=False,
                       recompute_scale_factor=False)[0, 0].numpy()
    return up[:h, :w]


def torch_sub(x, s, mode):
    """Subsample by s via torch on the largest divisible crop, then fill the
    ragged last row/column by the same rule applied to the clamped index."""
    h, w = x.shape
    hl, wl = -(-h // s), -(-w // s)
    out = np.empty((hl, wl))
    hd, wd = (h // s) * s, (w // s) * s
    if hd and wd:
        out[: h // s, : w // s] = (torch_nearest_sub if mode == "nearest" else torch_bilinear_sub)(
            x[:hd, :wd], s)
    # Ragged border: pad by edge replication to a divisible size and let torch
    # sample it; replication is what clamping taps to the image means.
    xp = np.pad(x, ((0, hl * s - h), (0, wl * s - w)), mode="edge")
    full = (torch_nearest_sub if mode == "nearest" else torch_bilinear_sub)(xp, s)
    out[h // s:, :] = full[h // s:, :]
    out[:, w // s:] = full[:, w // s:]
    return out


def composed_fast(I, p, r, s, eps, mode):
    """Algorithm 2 assembled from library primitives: torch subsample, scipy
    box means, numpy elementwise steps, torch upsample."""
    h, w = I.shape
    rl = 0 if r == 0 else max(1, int(math.floor(r / s + 0.5)))
    Il, pl = torch_sub(I, s, mode), torch_sub(p, s, mode)
    mI, mp = scipy_box(Il, rl), scipy_box(pl, rl)
    cI, cIp = scipy_box(Il * Il, rl), scipy_box(Il * pl, rl)
    a = (cIp - mI * mp) / (cI - mI * mI + eps)
    b = mp - a * mI
    ua = torch_upsample(scipy_box(a, rl), s, h, w)
    ub = torch_upsample(scipy_box(b, rl), s, h, w)
    return ua * I + ub


# ---------------------------------------------------------------- pins

def pin_lowres_rules(orc):
    """r' = r/s rounded half up (min 1 for r>0) and ceil(n/s) sizes."""
    table = {(8, 4): 2, (16, 4): 4, (32, 8): 4, (10, 4): 3, (3, 8): 1, (0, 4): 0, (5, 1): 5,
             (60, 4): 15, (4, 4): 1, (2, 4): 1, (6, 4): 2, (1, 1): 1, (7, 2): 4, (9, 8): 1}
    for (r, s), exp in table.items():
        assert orc.lowres_radius(r, s) == exp, (r, s, orc.lowres_radius(r, s), exp)
    for n, s, exp in [(512, 4, 128), (3000, 4, 750), (10, 4, 3), (1, 8, 1), (9, 8, 2), (7, 1, 7)]:
        assert orc.lowres_size(n, s) == exp, (n, s)


def pin_box_bruteforce(orc):
    """Box mean equals the literal clipped-window average (bit-exact on k/256 data)."""
    g = _rng(11)
    for h, w in [(1, 1), (1, 7), (6, 1), (3, 5), (8, 8), (12, 9), (5, 12)]:
        x = _dyadic(g, (h, w))
        for r in [0, 1, 2, 3, 6, 13]:
            exp = np.empty_like(x)
            for y in range(h):
                y0, y1 = _window(h, y, r)
                for xx in range(w):
                    x0, x1 = _window(w, xx, r)
                    blk = x[y0:y1 + 1, x0:x1 + 1]
                    exp[y, xx] = blk.sum() / blk.size
            got = orc.box_mean(x, r)
            assert np.array_equal(got, exp), (h, w, r, np.max(np.abs(got - exp)))


def pin_box_scipy(orc):
    """Box mean equals scipy's zero-padded uniform filter normalised by that of ones."""
    g = _rng(12)
    x = g.uniform(-1, 2, size=(41, 57))
    for r in [0, 1, 3, 10, 30, 70]:
        _close(orc.box_mean(x, r), scipy_box(x, r), 1e-12, f"box r={r}")


def pin_coefficients_lstsq(orc):
    """a_k, b_k minimise sum_{i in w_k} (a I_i + b - p_i)^2 + |w_k| eps a^2
    (the ridge regression whose normal equations are Eqs. 2-3)."""
    g = _rng(13)
    h, w = 9, 11
    I = g.uniform(0, 1, size=(h, w))
    p = 0.7 * I + g.uniform(0, 0.5, size=(h, w))
    for r, eps in [(1, 1e-2), (2, 0.3), (4, 1e-3)]:
        a, b = orc.coefficients(I, p, r, eps)
        for ky in range(h):
            y0, y1 = _window(h, ky, r)
            for kx in range(w):
                x0, x1 = _window(w, kx, r)
                Iw = I[y0:y1 + 1, x0:x1 + 1].ravel()
                pw = p[y0:y1 + 1, x0:x1 + 1].ravel()
                n = Iw.size
                A = np.vstack([np.stack([Iw, np.ones(n)], 1), [[math.sqrt(n * eps), 0.0]]])
                rhs = np.concatenate([pw, [0.0]])
                sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
                assert abs(a[ky, kx] - sol[0]) < 1e-10, (r, eps, ky, kx, a[ky, kx], sol[0])
                assert abs(b[ky, kx] - sol[1]) < 1e-10, (r, eps, ky, kx, b[ky, kx], sol[1])


def pin_eq4_average(orc):
    """Eq. 4: mean_a(i), mean_b(i) average a_k, b_k over every window k that
    contains i, and q_i = mean_a(i) I_i + mean_b(i)."""
    g = _rng(14)
    h, w, r, eps = 7, 10, 2, 0.05
    I = g.uniform(0, 1, size=(h, w))
    p = g.uniform(0, 1, size=(2, h, w))
    q, ex = orc.guided_filter(I, p, r, eps, intermediates=True)
    for c in range(2):
        a, b = orc.coefficients(I, p[c], r, eps)
        _close(ex["a"][c], a, 0.0, "a")
        for iy in range(h):
            for ix in range(w):
                ks = [(ky, kx) for ky in range(h) for kx in range(w)
                      if abs(ky - iy) <= r and abs(kx - ix) <= r]
                ma = sum(a[k] for k in ks) / len(ks)
                mb = sum(b[k] for k in ks) / len(ks)
                assert abs(ex["mean_a"][c, iy, ix] - ma) < 1e-13
                assert abs(ex["mean_b"][c, iy, ix] - mb) < 1e-13
                assert abs(q[c, iy, ix] - (ma * I[iy, ix] + mb)) < 1e-13


def pin_subsample_torch(orc):
    """Nearest = torch 'nearest-exact' (index s*y + floor(s/2)); bilinear =
    torch bilinear without antialias; ragged borders clamp to the image."""
    g = _rng(15)
    for h, w in [(16, 24), (13, 10), (9, 17), (1, 9)]:
        x = g.uniform(0, 1, size=(h, w))
        for s in [1, 2, 3, 4, 5, 8]:
            for mode in ("nearest", "bilinear"):
                _close(orc.subsample(x, s, mode), torch_sub(x, s, mode), 1e-15,
                       f"subsample {mode} s={s} {h}x{w}")


def pin_upsample_torch(orc):
    """Upsample = torch bilinear x s (half-pixel centres), cropped to h x w."""
    g = _rng(16)
    for (h, w), s in [((16, 12), 4), ((10, 7), 4), ((9, 13), 2), ((11, 6), 3), ((17, 8), 8),
                      ((1, 10), 4), ((5, 5), 1)]:
        lo = g.uniform(-1, 1, size=(-(-h // s), -(-w // s)))
        _close(orc.upsample(lo, s, h, w), torch_upsample(lo, s, h, w), 1e-14,
               f"upsample s={s} {h}x{w}")


def pin_composition(orc):
    """The whole fast filter equals Algorithm 2 assembled from library routines."""
    g = _rng(17)
    for (h, w), r, s, eps, mode in [((37, 45), 8, 4, 1e-2, "nearest"),
                                    ((37, 45), 8, 4, 1e-2, "bilinear"),
                                    ((30, 21), 5, 2, 1e-3, "nearest"),
                                    ((29, 33), 6, 3, 1e-1, "bilinear"),
                                    ((40, 40), 3, 1, 1e-2, "nearest")]:
        I = g.uniform(0, 1, size=(h, w))
        p = np.clip(I + g.normal(0, 0.1, size=(h, w)), 0, 1)
        _close(orc.fast_guided_filter(I, p, r, s, eps, mode), composed_fast(I, p, r, s, eps, mode),
               1e-11, f"fast {h}x{w} r={r} s={s} {mode}")


def pin_bruteforce_eqs(orc):
    """Eqs. 2-4 by explicit per-window loops (no box filter) on tiny images."""
    g = _rng(18)
    h, w, r, eps = 6, 8, 2, 0.02
    I = g.uniform(0, 1, size=(h, w))
    p = g.uniform(0, 1, size=(h, w))
    a = np.empty((h, w))
    b = np.empty((h, w))
    for ky in range(h):
        for kx in range(w):
            pts = [(y, x) for y in range(h) for x in range(w) if abs(y - ky) <= r and abs(x - kx) <= r]
            n = len(pts)
            mu = sum(I[t] for t in pts) / n
            pbar = sum(p[t] for t in pts) / n
            var = sum((I[t] - mu) ** 2 for t in pts) / n
            a[ky, kx] = (sum(I[t] * p[t] for t in pts) / n - mu * pbar) / (var + eps)
            b[ky, kx] = pbar - a[ky, kx] * mu
    q = np.empty((h, w))
    for iy in range(h):
        for ix in range(w):
            ks = [(y, x) for y in range(h) for x in range(w) if abs(y - iy) <= r and abs(x - ix) <= r]
            q[iy, ix] = sum(a[k] * I[iy, ix] + b[k] for k in ks) / len(ks)
    _close(orc.guided_filter(I, p, r, eps), q, 1e-13, "brute-force Eqs. 2-4")


def pin_constant_input(orc):
    """p constant => q equals that constant (a = 0, b = p)."""
    g = _rng(19)
    I = g.uniform(0, 1, size=(23, 31))
    for cval, tol in [(0.5, 0.0), (0.3, 1e-15)]:
        p = np.full_like(I, cval)
        _close(orc.guided_filter(I, p, 4, 1e-3), p, tol, "plain const p")
        for mode in ("nearest", "bilinear"):
            _close(orc.fast_guided_filter(I, p, 8, 4, 1e-3, mode), p, tol, "fast const p")


def pin_constant_guide(orc):
    """I constant => var = cov = 0, a = 0, and q = up(B(B(p'))): the input
    box-filtered twice at the low-res radius, then upsampled."""
    g = _rng(20)
    h, w = 26, 35
    I = np.full((h, w), 0.5)
    p = g.uniform(0, 1, size=(h, w))
    _, ex = orc.guided_filter(I, p, 3, 1e-3, intermediates=True)
    assert np.all(ex["a"] == 0.0)
    _close(orc.guided_filter(I, p, 3, 1e-3), scipy_box(scipy_box(p, 3), 3), 1e-14, "plain const I")
    for s, r, mode in [(4, 8, "nearest"), (2, 3, "bilinear"), (3, 7, "nearest")]:
        rl = max(1, int(math.floor(r / s + 0.5)))
        exp = torch_upsample(scipy_box(scipy_box(torch_sub(p, s, mode), rl), rl), s, h, w)
        _close(orc.fast_guided_filter(I, p, r, s, 1e-3, mode), exp, 1e-14, f"fast const I s={s}")


def pin_fast_s1_is_plain(orc):
    """At s = 1 subsample and upsample are identities: fast == plain bit for bit."""
    g = _rng(21)
    I = g.uniform(0, 1, size=(19, 27))
    p = g.uniform(0, 1, size=(3, 19, 27))
    for mode in ("nearest", "bilinear"):
        assert np.array_equal(orc.fast_guided_filter(I, p, 4, 1, 1e-2, mode),
                              orc.guided_filter(I, p, 4, 1e-2))


def pin_r0_identity(orc):
    """r = 0: every window is one pixel, var = cov = 0, so q = p exactly."""
    g = _rng(22)
    I = g.uniform(0, 1, size=(9, 14))
    p = g.uniform(0, 1, size=(9, 14))
    assert np.array_equal(orc.guided_filter(I, p, 0, 1e-3), p)
    assert np.array_equal(orc.fast_guided_filter(I, p, 0, 1, 1e-3), p)


def pin_linearity(orc):
    """q is linear in p: q(al p1 + be p2) = al q(p1) + be q(p2)."""
    g = _rng(23)
    I = g.uniform(0, 1, size=(33, 29))
    p1, p2 = g.uniform(0, 1, size=(2, 33, 29))
    lhs = orc.fast_guided_filter(I, 0.7 * p1 - 1.3 * p2, 6, 2, 1e-2, "bilinear")
    rhs = 0.7 * orc.fast_guided_filter(I, p1, 6, 2, 1e-2, "bilinear") - 1.3 * orc.fast_guided_filter(
        I, p2, 6, 2, 1e-2, "bilinear")
    _close(lhs, rhs, 1e-13, "linearity")


def pin_offset(orc):
    """q(I, p + c) = q(I, p) + c (needs the clip normalisation to be a mean)."""
    g = _rng(24)
    I = g.uniform(0, 1, size=(31, 22))
    p = g.uniform(0, 1, size=(31, 22))
    _close(orc.guided_filter(I, p + 0.25, 5, 1e-2), orc.guided_filter(I, p, 5, 1e-2) + 0.25,
           1e-14, "offset plain")
    _close(orc.fast_guided_filter(I, p + 0.25, 9, 4, 1e-2),
           orc.fast_guided_filter(I, p, 9, 4, 1e-2) + 0.25, 1e-14, "offset fast")


def pin_guide_shift_scale(orc):
    """q(I + c, p) = q(I, p); q(2 I, p; 4 eps) = q(I, p; eps) bit for bit."""
    g = _rng(25)
    I = g.uniform(0, 1, size=(27, 30))
    p = g.uniform(0, 1, size=(27, 30))
    base = orc.fast_guided_filter(I, p, 6, 2, 1e-2)
    _close(orc.fast_guided_filter(I + 0.375, p, 6, 2, 1e-2), base, 1e-13, "guide shift")
    assert np.array_equal(orc.fast_guided_filter(2 * I, p, 6, 2, 4e-2), base)
    assert np.array_equal(orc.guided_filter(2 * I, p, 3, 4e-2), orc.guided_filter(I, p, 3, 1e-2))


def pin_affine_reproduction(orc):
    """Eq. 1: if p = al I + be and eps -> 0 (no flat window), a = al and
    b = be everywhere, so q = al I + be for the plain and the fast filter
    (the output uses the full-resolution I)."""
    g = _rng(26)
    I = g.uniform(0, 1, size=(41, 38))
    p = 0.8 * I + 0.1
    _close(orc.guided_filter(I, p, 3, 1e-14), p, 1e-8, "affine plain")
    for s, mode in [(4, "nearest"), (2, "bilinear"), (3, "nearest")]:
        _close(orc.fast_guided_filter(I, p, 8, s, 1e-14, mode), p, 1e-8, f"affine fast s={s}")


def pin_large_eps(orc):
    """eps -> infinity: a -> 0 and q -> up(B(B(p'))) as for a constant guide."""
    g = _rng(27)
    h, w = 24, 28
    I = g.uniform(0, 1, size=(h, w))
    p = g.uniform(0, 1, size=(h, w))
    exp = torch_upsample(scipy_box(scipy_box(torch_sub(p, 4, "nearest"), 2), 2), 4, h, w)
    _close(orc.fast_guided_filter(I, p, 8, 4, 1e30), exp, 1e-12, "large eps")


def pin_transpose(orc):
    """Transposing I and p transposes q."""
    g = _rng(28)
    I = g.uniform(0, 1, size=(21, 34))
    p = g.uniform(0, 1, size=(21, 34))
    for s, mode in [(1, "nearest"), (4, "nearest"), (2, "bilinear")]:
        _close(orc.fast_guided_filter(I.T, p.T, 7, s, 1e-2, mode),
               orc.fast_guided_filter(I, p, 7, s, 1e-2, mode).T, 1e-14, f"transpose s={s}")


def pin_degenerate_shapes(orc):
    """1xN, Nx1, sizes not divisible by s, and r' larger than the low-res map."""
    g = _rng(29)
    for (h, w), r, s, mode in [((1, 37), 4, 4, "nearest"), ((29, 1), 6, 2, "bilinear"),
                               ((7, 9), 40, 4, "nearest"), ((3, 3), 9, 8, "bilinear"),
                               ((13, 18), 5, 3, "nearest"), ((1, 1), 2, 4, "nearest")]:
        I = g.uniform(0, 1, size=(h, w))
        p = g.uniform(0, 1, size=(h, w))
        _close(orc.fast_guided_filter(I, p, r, s, 1e-2, mode), composed_fast(I, p, r, s, 1e-2, mode),
               1e-11, f"degenerate {h}x{w} r={r} s={s}")


def composed_joint(I, p_lo, r, s, eps, mode):
    """Joint upsampling assembled from library primitives: torch subsample of
    the guide only, scipy box means, numpy elementwise steps, torch upsample."""
    h, w = I.shape
    rl = 0 if r == 0 else max(1, int(math.floor(r / s + 0.5)))
    Il = torch_sub(I, s, mode)
    mI, mp = scipy_box(Il, rl), scipy_box(p_lo, rl)
    cI, cIp = scipy_box(Il * Il, rl), scipy_box(Il * p_lo, rl)
    a = (cIp - mI * mp) / (cI - mI * mI + eps)
    b = mp - a * mI
    return torch_upsample(scipy_box(a, rl), s, h, w) * I + torch_upsample(scipy_box(b, rl), s, h, w)


def pin_joint_composition(orc):
    """Joint upsampling equals its assembly from library routines, for a
    low-res input that is not a subsampled full-res image."""
    g = _rng(31)
    for (h, w), r, s, eps, mode in [((37, 45), 8, 4, 1e-2, "nearest"), ((30, 21), 5, 2, 1e-3, "bilinear"),
                                    ((29, 33), 6, 3, 1e-1, "nearest"), ((8, 50), 12, 8, 1e-2, "bilinear")]:
        I = g.uniform(0, 1, size=(h, w))
        p_lo = g.uniform(0, 1, size=(-(-h // s), -(-w // s)))
        _close(orc.joint_upsample(I, p_lo, r, s, eps, mode), composed_joint(I, p_lo, r, s, eps, mode), 1e-11,
               f"joint {h}x{w} r={r} s={s} {mode}")


def pin_joint_of_subsampled_is_fast(orc):
    """Given p subsampled by the library routine, joint upsampling is the fast
    filter of the full-resolution p (every channel)."""
    g = _rng(32)
    for (h, w), r, s, mode in [((33, 40), 8, 4, "nearest"), ((26, 31), 4, 2, "bilinear")]:
        I = g.uniform(0, 1, size=(h, w))
        p = g.uniform(0, 1, size=(2, h, w))
        p_lo = np.stack([torch_sub(p[k], s, mode) for k in range(2)])
        _close(orc.joint_upsample(I, p_lo, r, s, 1e-2, mode), orc.fast_guided_filter(I, p, r, s, 1e-2, mode),
               1e-13, f"joint of subsampled p {h}x{w} s={s} {mode}")


def pin_joint_constant(orc):
    """A constant low-res input comes back as that constant at full resolution."""
    g = _rng(33)
    I = g.uniform(0, 1, size=(21, 34))
    for mode in ("nearest", "bilinear"):
        _close(orc.joint_upsample(I, np.full((6, 9), 0.5), 8, 4, 1e-3, mode), np.full((21, 34), 0.5), 0.0,
               f"joint const {mode}")


def pin_detail_gain_endpoints(orc):
    """Detail enhancement with gain 0 is the filtered image, with gain 1 the
    input; a constant input is unchanged at any gain."""
    g = _rng(34)
    I = g.uniform(0, 1, size=(17, 23))
    p = np.clip(I + g.normal(0, 0.1, size=(17, 23)), 0, 1)
    q = orc.fast_guided_filter(I, p, 8, 4, 1e-2)
    assert np.array_equal(orc.detail_enhance(p, q, 0.0), q)
    _close(orc.detail_enhance(p, q, 1.0), p, 2e-16, "gain 1")
    c = np.full_like(p, 0.25)
    _close(orc.detail_enhance(c, orc.fast_guided_filter(I, c, 8, 4, 1e-2), 5.0), c, 1e-15, "constant input")


def pin_detail_gain5_hand(orc):
    """The paper's x5 detail on values worked by hand: base q, detail p - q,
    e = q + 5 (p - q).  (p, q) = (0.75, 0.5) gives 0.5 + 1.25 = 1.75;
    (0.25, 0.5) gives 0.5 - 1.25 = -0.75; p = q gives q; (0, 0.125) gives
    0.125 - 0.625 = -0.5.  All dyadic, so the results are exact."""
    p = np.array([[0.75, 0.25], [0.5, 0.0]])
    q = np.array([[0.5, 0.5], [0.5, 0.125]])
    assert np.array_equal(orc.detail_enhance(p, q, 5.0), [[1.75, -0.75], [0.5, -0.5]])


# ---------------------------------------------------------------- borders and area subsampling

_NP_PAD = {"replicate": "edge", "reflect101": "reflect"}     # numpy's names for the same extensions
_SCIPY_MODE = {"replicate": "nearest", "reflect101": "mirror"}


def padded_window_mean(x, r, border):
    """Literal mean of every (2r+1)^2 window of the image padded by numpy."""
    from numpy.lib.stride_tricks import sliding_window_view
    xp = np.pad(np.asarray(x, dtype=np.float64), r, mode=_NP_PAD[border])
    return sliding_window_view(xp, (2 * r + 1, 2 * r + 1)).mean(axis=(-1, -2))


def lib_box(x, r, border):
    """Box mean by scipy: clip-normalised, or its uniform filter in the padded modes."""
    if border == "clip":
        return scipy_box(x, r)
    return ndi.uniform_filter(np.asarray(x, dtype=np.float64), size=2 * r + 1, mode=_SCIPY_MODE[border])


def torch_area_sub(x, s):
    """Mean of each s x s block (blocks at a ragged edge averaged over their in-image part)."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))[None, None]
    return F.avg_pool2d(t, kernel_size=s, stride=s, ceil_mode=True)[0, 0].numpy()


def lib_sub(x, s, mode):
    return torch_area_sub(x, s) if mode == "area" else torch_sub(x, s, mode)


def composed_general(I, p_lo, r, s, eps, mode, border, joint=False):
    """Algorithm 2 from library routines for any subsampling and border:
    torch subsampling (or average pooling), scipy box means, torch upsample.
    With joint, p_lo is the low-res input and only I is subsampled."""
    h, w = I.shape
    rl = 0 if r == 0 else max(1, int(math.floor(r / s + 0.5)))
    Il = lib_sub(I, s, mode) if s > 1 else I
    pl = p_lo if (joint or s == 1) else lib_sub(p_lo, s, mode)
    mI, mp = lib_box(Il, rl, border), lib_box(pl, rl, border)
    cI, cIp = lib_box(Il * Il, rl, border), lib_box(Il * pl, rl, border)
    a = (cIp - mI * mp) / (cI - mI * mI + eps)
    b = mp - a * mI
    ma, mb = lib_box(a, rl, border), lib_box(b, rl, border)
    if s == 1:
        return ma * I + mb
    return torch_upsample(ma, s, h, w) * I + torch_upsample(mb, s, h, w)


def pin_box_padded_numpy(orc):
    """Padded box means equal the literal window mean over numpy's edge /
    reflect padding, also for windows wider than the image (repeated
    reflection) and one-pixel axes."""
    g = _rng(41)
    for h, w in [(1, 1), (1, 7), (6, 1), (3, 5), (8, 8), (12, 9), (2, 2)]:
        x = _dyadic(g, (h, w))
        for r in [0, 1, 2, 5, 13]:
            for border in ("replicate", "reflect101"):
                _close(orc.box_mean(x, r, border), padded_window_mean(x, r, border), 4e-16,
                       f"padded box {border} {h}x{w} r={r}")


def pin_box_padded_scipy(orc):
    """Padded box means equal scipy's uniform filter in 'nearest' (replicate)
    and 'mirror' (reflect-101) modes."""
    g = _rng(42)
    x = g.uniform(-1, 2, size=(23, 31))
    for r in [1, 4, 11, 40]:
        for border in ("replicate", "reflect101"):
            _close(orc.box_mean(x, r, border), lib_box(x, r, border), 1e-12, f"scipy box {border} r={r}")


def pin_area_subsample_pool(orc):
    """Area subsampling equals torch's average pooling with an s x s window and
    stride s (ceil mode: the ragged last block is averaged over its in-image
    part), and a reshape-mean when s divides the sides."""
    g = _rng(43)
    for h, w in [(16, 24), (13, 10), (9, 17), (1, 9), (7, 1)]:
        x = g.uniform(0, 1, size=(h, w))
        for s in [1, 2, 3, 4, 5, 8]:
            _close(orc.subsample(x, s, "area"), torch_area_sub(x, s), 1e-15, f"area s={s} {h}x{w}")
    x = g.uniform(0, 1, size=(24, 32))
    _close(orc.subsample(x, 4, "area"), x.reshape(6, 4, 8, 4).mean(axis=(1, 3)), 1e-15, "area reshape")


def pin_border_area_composition(orc):
    """The plain and fast filters and joint upsampling under every border and
    subsampling convention equal their assembly from library routines."""
    g = _rng(44)
    cases = [((37, 45), 8, 4, 1e-2, "nearest", "replicate"), ((37, 45), 8, 4, 1e-2, "bilinear", "reflect101"),
             ((30, 21), 5, 2, 1e-3, "area", "clip"), ((29, 33), 6, 3, 1e-1, "area", "reflect101"),
             ((13, 50), 12, 4, 1e-2, "area", "replicate"), ((40, 40), 3, 1, 1e-2, "nearest", "reflect101"),
             ((9, 11), 6, 1, 1e-2, "nearest", "replicate"), ((10, 12), 24, 8, 1e-2, "nearest", "reflect101")]
    for (h, w), r, s, eps, mode, border in cases:
        I = g.uniform(0, 1, size=(h, w))
        p = np.clip(I + g.normal(0, 0.1, size=(h, w)), 0, 1)
        what = f"{h}x{w} r={r} s={s} {mode} {border}"
        _close(orc.fast_guided_filter(I, p, r, s, eps, mode, border=border),
               composed_general(I, p, r, s, eps, mode, border), 1e-11, "fast " + what)
        if s == 1:
            _close(orc.guided_filter(I, p, r, eps, border=border), composed_general(I, p, r, 1, eps, mode, border),
                   1e-11, "plain " + what)
        else:
            p_lo = g.uniform(0, 1, size=(-(-h // s), -(-w // s)))
            _close(orc.joint_upsample(I, p_lo, r, s, eps, mode, border=border),
                   composed_general(I, p_lo, r, s, eps, mode, border, joint=True), 1e-11, "joint " + what)


def pin_padded_coefficients_lstsq(orc):
    """With a padded border, a_k, b_k solve the ridge regression over the
    (2r+1)^2 samples of the padded window (edge samples counted as often as
    the padding repeats them)."""
    g = _rng(45)
    h, w = 6, 7
    I = g.uniform(0, 1, size=(h, w))
    p = 0.6 * I + g.uniform(0, 0.5, size=(h, w))
    for border in ("replicate", "reflect101"):
        for r, eps in [(1, 1e-2), (3, 0.2), (8, 1e-3)]:
            _, ex = orc.guided_filter(I, p, r, eps, intermediates=True, border=border)
            Ip, pp = np.pad(I, r, mode=_NP_PAD[border]), np.pad(p, r, mode=_NP_PAD[border])
            n = (2 * r + 1) ** 2
            for ky, kx in [(0, 0), (0, w - 1), (h - 1, 3), (2, 3), (h - 1, w - 1)]:
                Iw = Ip[ky:ky + 2 * r + 1, kx:kx + 2 * r + 1].ravel()
                pw = pp[ky:ky + 2 * r + 1, kx:kx + 2 * r + 1].ravel()
                A = np.vstack([np.stack([Iw, np.ones(n)], 1), [[math.sqrt(n * eps), 0.0]]])
                sol = np.linalg.lstsq(A, np.concatenate([pw, [0.0]]), rcond=None)[0]
                assert abs(ex["a"][ky, kx] - sol[0]) < 1e-10, (border, r, ky, kx, ex["a"][ky, kx], sol[0])
                assert abs(ex["b"][ky, kx] - sol[1]) < 1e-10, (border, r, ky, kx, ex["b"][ky, kx], sol[1])


def pin_border_constant(orc):
    """A constant input is returned exactly under every border; with a
    constant guide, q is the border's box mean of the box mean of p."""
    g = _rng(46)
    I = g.uniform(0, 1, size=(19, 26))
    for border in ("replicate", "reflect101"):
        for mode in ("nearest", "area"):
            _close(orc.fast_guided_filter(I, np.full((19, 26), 0.375), 8, 4, 1e-3, mode, border=border),
                   np.full((19, 26), 0.375), 1e-14, f"constant p {border} {mode}")
        p = g.uniform(0, 1, size=(19, 26))
        exp = padded_window_mean(padded_window_mean(p, 3, border), 3, border)
        _close(orc.guided_filter(np.full((19, 26), 0.5), p, 3, 1e-2, border=border), exp, 1e-14,
               f"constant guide {border}")


# ---------------------------------------------------------------- colour guidance

def _windows(n, i, r, border):
    """Indices along an axis that the window of radius r at i reads."""
    if border == "clip":
        return list(range(max(0, i - r), min(n - 1, i + r) + 1))
    idx = np.pad(np.arange(n), r, mode=_NP_PAD[border])
    return list(idx[i:i + 2 * r + 1])


def pin_color_coefficients_lstsq(orc):
    """a_k (3-vector), b_k minimise sum_{i in w_k} (a.I_i + b - p_i)^2 + |w_k| eps |a|^2
    over the window's samples (clip-normalised and padded windows)."""
    g = _rng(51)
    h, w = 7, 9
    I = g.uniform(0, 1, size=(3, h, w))
    p = 0.3 * I[0] - 0.2 * I[1] + 0.5 * I[2] + g.uniform(0, 0.3, size=(h, w))
    for border in ("clip", "replicate", "reflect101"):
        for r, eps in [(1, 1e-2), (2, 0.2), (4, 1e-3)]:
            _, ex = orc.fast_guided_filter_color(I, p, r, 1, eps, border=border, intermediates=True)
            for ky, kx in [(0, 0), (0, w - 1), (h - 1, 4), (3, 4), (h - 1, w - 1), (2, 0)]:
                ys, xs = _windows(h, ky, r, border), _windows(w, kx, r, border)
                Iw = np.stack([I[j][np.ix_(ys, xs)].ravel() for j in range(3)], 1)
                pw = p[np.ix_(ys, xs)].ravel()
                n = pw.size
                A = np.vstack([np.hstack([Iw, np.ones((n, 1))]),
                               np.hstack([math.sqrt(n * eps) * np.eye(3), np.zeros((3, 1))])])
                sol = np.linalg.lstsq(A, np.concatenate([pw, np.zeros(3)]), rcond=None)[0]
                assert np.allclose(ex["a"][:, ky, kx], sol[:3], atol=1e-9, rtol=0), (border, r, ky, kx)
                assert abs(ex["b"][ky, kx] - sol[3]) < 1e-9, (border, r, ky, kx)


def composed_color(I, p, r, s, eps, mode, border, joint=False):
    """Colour guidance from library routines: torch subsampling (or pooling),
    scipy box means, numpy's batched 3x3 solve, torch upsampling.  With
    joint, p is the low-res input and only the guide is subsampled."""
    h, w = I.shape[1:]
    rl = 0 if r == 0 else max(1, int(math.floor(r / s + 0.5)))
    Il = np.stack([lib_sub(I[j], s, mode) if s > 1 else I[j] for j in range(3)])
    pl = p if (joint or s == 1) else lib_sub(p, s, mode)
    mI = np.stack([lib_box(Il[j], rl, border) for j in range(3)])
    mp = lib_box(pl, rl, border)
    S = np.empty(Il.shape[1:] + (3, 3))
    for j in range(3):
        for k in range(3):
            S[..., j, k] = lib_box(Il[j] * Il[k], rl, border) - mI[j] * mI[k]
    S += eps * np.eye(3)
    cov = np.stack([lib_box(Il[j] * pl, rl, border) - mI[j] * mp for j in range(3)], -1)
    a = np.linalg.solve(S, cov[..., None])[..., 0]
    b = mp - np.einsum("...j,j...->...", a, mI)
    up = (lambda x: x) if s == 1 else (lambda x: torch_upsample(x, s, h, w))
    q = up(lib_box(b, rl, border))
    for j in range(3):
        q = q + up(lib_box(a[..., j], rl, border)) * I[j]
    return q


def pin_color_composition(orc):
    """The colour filter (plain and fast, every border and subsampling)
    equals its assembly from library routines."""
    g = _rng(52)
    for (h, w), r, s, eps, mode, border in [((23, 31), 4, 1, 1e-2, "nearest", "clip"),
                                            ((37, 45), 8, 4, 1e-2, "nearest", "clip"),
                                            ((30, 21), 5, 2, 1e-3, "bilinear", "reflect101"),
                                            ((29, 33), 6, 3, 1e-1, "area", "replicate"),
                                            ((12, 40), 12, 4, 1e-3, "nearest", "reflect101")]:
        I = g.uniform(0, 1, size=(3, h, w))
        p = np.clip(0.5 * I[0] + 0.3 * I[2] + g.normal(0, 0.1, size=(h, w)), 0, 1)
        _close(orc.fast_guided_filter_color(I, p, r, s, eps, mode, border), composed_color(I, p, r, s, eps, mode, border),
               1e-10, f"colour {h}x{w} r={r} s={s} {mode} {border}")


def pin_color_gray_guide(orc):
    """A guide of three equal planes G: the colour filter is the gray filter
    of G with eps/3 (Sigma = var 11^T, whose eigenvalue along (1,1,1) is
    3 var, so a = cov / (3 var + eps) (1,1,1))."""
    g = _rng(53)
    G = g.uniform(0, 1, size=(26, 34))
    p = g.uniform(0, 1, size=(2, 26, 34))
    for s, mode, border in [(1, "nearest", "clip"), (4, "nearest", "clip"), (2, "bilinear", "reflect101")]:
        _close(orc.fast_guided_filter_color(np.stack([G, G, G]), p, 6, s, 3e-2, mode, border),
               orc.fast_guided_filter(G, p, 6, s, 1e-2, mode, border=border), 1e-10, f"equal planes s={s}")


def pin_color_joint(orc):
    """Colour joint upsampling equals its library assembly for a low-res
    input that is not a subsample, and the colour fast filter when p_lo is
    p subsampled by the library routine."""
    g = _rng(55)
    for (h, w), r, s, mode, border in [((33, 40), 8, 4, "nearest", "clip"), ((26, 31), 4, 2, "bilinear", "reflect101"),
                                       ((30, 27), 6, 3, "area", "replicate")]:
        I = g.uniform(0, 1, size=(3, h, w))
        p_lo = g.uniform(0, 1, size=(-(-h // s), -(-w // s)))
        got = orc.joint_upsample_color(I, p_lo, r, s, 1e-2, mode, border)
        _close(got, composed_color(I, p_lo, r, s, 1e-2, mode, border, joint=True), 1e-10,
               f"colour joint {h}x{w} s={s} {mode} {border}")
        p = g.uniform(0, 1, size=(2, h, w))
        p_sub = np.stack([lib_sub(p[k], s, mode) for k in range(2)])
        _close(orc.joint_upsample_color(I, p_sub, r, s, 1e-2, mode, border),
               orc.fast_guided_filter_color(I, p, r, s, 1e-2, mode, border), 1e-13,
               f"colour joint of subsampled p s={s} {mode}")


def pin_color_invariants(orc):
    """Constant p returns p; adding a constant to a guide plane changes
    nothing; a p that is an affine function of the guide comes back as
    itself as eps -> 0; channels of p are independent."""
    g = _rng(54)
    I = g.uniform(0, 1, size=(3, 19, 23))
    _close(orc.fast_guided_filter_color(I, np.full((19, 23), 0.25), 5, 2, 1e-2), np.full((19, 23), 0.25), 1e-13,
           "constant p")
    p = g.uniform(0, 1, size=(19, 23))
    q = orc.fast_guided_filter_color(I, p, 5, 2, 1e-2)
    _close(orc.fast_guided_filter_color(I + np.array([0.3, -0.2, 0.1])[:, None, None], p, 5, 2, 1e-2),
           q, 1e-9, "guide offset")
    lin = 0.4 * I[0] - 0.7 * I[1] + 0.2 * I[2] + 0.1
    _close(orc.fast_guided_filter_color(I, lin, 3, 1, 1e-12), lin, 1e-7, "affine p")
    pp = g.uniform(0, 1, size=(2, 19, 23))
    both = orc.fast_guided_filter_color(I, pp, 4, 2, 1e-2)
    _close(both[1], orc.fast_guided_filter_color(I, pp[1], 4, 2, 1e-2), 0.0, "channel independence")


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
