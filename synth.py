"""Seeded synthetic inputs for the guided-filter tests and benchmark.

This module only draws images and request mixes (numpy PCG64); it holds none
of the filter's arithmetic, so both the GPU path and the FP64 oracle can be
fed from it.  The paper's own photographs are not available; these stand in
for them with the shapes and value ranges of its workloads: [0, 1] images,
piecewise-smooth guides with sharp edges, colour inputs correlated with the
guide, and near-flat regions that stress the variance term.

Every generator returns float32 arrays (the 16-bit variants are made by the
caller with a round-to-nearest-even cast).  Images are (H, W) for the guide
and (C, H, W) for the filtering input.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def rectangles(h: int, w: int, seed: int = 0, noise: float = 0.05) -> np.ndarray:
    """Piecewise-constant guide: uniform background with random 8-32 px
    rectangles of uniform value, plus Gaussian noise, clipped to [0, 1]."""
    g = _rng(seed)
    img = np.full((h, w), g.uniform(0.0, 1.0), dtype=np.float64)
    n_rect = math.ceil(2 * h * w / 20 ** 2)
    for _ in range(n_rect):
        rh, rw = g.integers(8, 33, size=2)
        y0, x0 = g.integers(0, max(1, h - 1)), g.integers(0, max(1, w - 1))
        img[y0:y0 + rh, x0:x0 + rw] = g.uniform(0.0, 1.0)
    img += g.normal(0.0, noise, size=(h, w))
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def noisy_copy(I: np.ndarray, seed: int, sigma: float = 0.1) -> np.ndarray:
    """p = clip(I + N(0, sigma^2)) with noise independent of the guide's."""
    g = _rng(seed)
    return np.clip(I.astype(np.float64) + g.normal(0.0, sigma, size=I.shape), 0.0, 1.0).astype(np.float32)


def _grid(h: int, w: int):
    y = (np.arange(h, dtype=np.float32) + 0.5) / h
    x = (np.arange(w, dtype=np.float32) + 0.5) / w
    return y[:, None], x[None, :]


def _smooth_field(g: np.random.Generator, h: int, w: int, terms: int, amp: float) -> np.ndarray:
    """Sum of low-frequency cosines (at most 3 cycles across the image)."""
    y, x = _grid(h, w)
    out = np.zeros((h, w), dtype=np.float32)
    for _ in range(terms):
        fy, fx = g.uniform(0.0, 3.0, size=2)
        ph = g.uniform(0.0, 2 * math.pi)
        a = g.uniform(0.0, amp)
        out += np.float32(a) * np.cos(np.float32(2 * math.pi) * (np.float32(fy) * y + np.float32(fx) * x)
                                      + np.float32(ph))
    return out


def _steps(g: np.random.Generator, h: int, w: int, n: int) -> np.ndarray:
    """n random half-plane or disc steps of height +-U[0.1, 0.3]."""
    y, x = _grid(h, w)
    out = np.zeros((h, w), dtype=np.float32)
    for _ in range(n):
        height = np.float32(g.choice([-1.0, 1.0]) * g.uniform(0.1, 0.3))
        cy, cx = g.uniform(0.0, 1.0, size=2)
        if g.uniform() < 0.5:
            th = g.uniform(0.0, 2 * math.pi)
            mask = (np.float32(math.cos(th)) * (x - np.float32(cx))
                    + np.float32(math.sin(th)) * (y - np.float32(cy))) > 0
        else:
            rad = g.uniform(0.05, 0.3)
            mask = ((x - np.float32(cx)) ** 2 + (y - np.float32(cy)) ** 2) < np.float32(rad * rad)
        out += height * mask
    return out


def photo_guide(h: int, w: int, seed: int, noise: float = 0.02) -> np.ndarray:
    """Gray guide: 0.5 + smooth gradients + 16 edges + N(0, noise^2), clipped."""
    g = _rng(seed)
    I = np.float32(0.5) + _smooth_field(g, h, w, 4, 0.15) + _steps(g, h, w, 16)
    I += g.standard_normal(size=(h, w), dtype=np.float32) * np.float32(noise)
    return np.clip(I, 0.0, 1.0)


def colour_input(I: np.ndarray, c: int, seed: int, noise: float = 0.05) -> np.ndarray:
    """p_c = clip(g_c I + o_c + smooth colour field_c + N(0, noise^2)), g_c in [0.6, 1.2]."""
    g = _rng(seed)
    h, w = I.shape
    out = np.empty((c, h, w), dtype=np.float32)
    for k in range(c):
        gain = np.float32(g.uniform(0.6, 1.2))
        off = np.float32(g.uniform(-0.1, 0.1))
        pk = gain * I + off + _smooth_field(g, h, w, 2, 0.1)
        pk += g.standard_normal(size=(h, w), dtype=np.float32) * np.float32(noise)
        out[k] = np.clip(pk, 0.0, 1.0)
    return out


def colour_guide(h: int, w: int, seed: int, noise: float = 0.02) -> np.ndarray:
    """Three-channel guide (3, h, w): a shared photo-like luminance G with,
    per channel, gain in [0.7, 1.1], offset in [-0.1, 0.1], a smooth tint
    field and N(0, noise^2), clipped to [0, 1]."""
    g = _rng(seed)
    G = photo_guide(h, w, seed + 1000, noise)
    out = np.empty((3, h, w), dtype=np.float32)
    for k in range(3):
        gain = np.float32(g.uniform(0.7, 1.1))
        off = np.float32(g.uniform(-0.1, 0.1))
        ck = gain * G + off + _smooth_field(g, h, w, 3, 0.1)
        ck += g.standard_normal(size=(h, w), dtype=np.float32) * np.float32(noise)
        out[k] = np.clip(ck, 0.0, 1.0)
    return out


def flat_blocks_guide(h: int, w: int, seed: int, block: int = 500) -> np.ndarray:
    """Guide whose blocks are, with probability 1/2, near-constant in
    [0.49, 0.51] (0.5 + 0.01 * smooth field); the rest is photo content."""
    g = _rng(seed)
    I = photo_guide(h, w, seed + 1000)
    flat = np.float32(0.5) + np.float32(0.01) * np.clip(_smooth_field(g, h, w, 3, 1.0) / 3.0, -1, 1)
    for by in range(0, h, block):
        for bx in range(0, w, block):
            if g.uniform() < 0.5:
                I[by:by + block, bx:bx + block] = flat[by:by + block, bx:bx + block]
    return I


# --- the named workloads -------------------------------------------------

def workload_small(seed_I: int = 0, seed_p: int = 1, h: int = 512, w: int = 512):
    """512x512 gray guide and gray input (rectangles + noise); r=8, s=4, eps=0.01."""
    I = rectangles(h, w, seed_I)
    p = noisy_copy(I, seed_p)
    return I, p[None]


def workload_12mp(h: int = 3000, w: int = 4000, c: int = 3, seed_I: int = 2, seed_p: int = 3):
    """4000x3000 gray guide, RGB input; r=16, s=4 (and s=1), eps=1e-3."""
    I = photo_guide(h, w, seed_I)
    return I, colour_input(I, c, seed_p)


def workload_12mp_colour(h: int = 3000, w: int = 4000, c: int = 3, seed_I: int = 6, seed_p: int = 7):
    """4000x3000 RGB guide, RGB input (p from the guide's mean luminance)."""
    I = colour_guide(h, w, seed_I)
    return I, colour_input(I.mean(axis=0, dtype=np.float32), c, seed_p)


def workload_24mp(h: int = 4000, w: int = 6000, c: int = 3, seed_I: int = 4, seed_p: int = 5):
    """6000x4000 guide with near-flat blocks, RGB input; r=32, s=8, eps 1e-4 / 1e-6."""
    I = flat_blocks_guide(h, w, seed_I)
    return I, colour_input(I, c, seed_p)


@dataclass
class ImageSpec:
    h: int
    w: int
    c: int
    r: int
    s: int
    eps: float
    seed: int


def radius_for(h: int, w: int) -> int:
    """Filter radius proportional to image size: round(0.01 * max(H, W))."""
    return (max(h, w) + 50) // 100


def batch_specs(n: int = 256, seed: int = 6, hmax: int = 1536, wmax: int = 2048) -> list[ImageSpec]:
    """Uneven batch: H~U{256..hmax}, W~U{256..wmax}, swapped with prob. 1/2,
    r = round(0.01 max(H, W)), s in {2,4,8}, C in {1,3}, eps = 1e-3."""
    g = _rng(seed)
    specs = []
    for i in range(n):
        h, w = int(g.integers(256, hmax + 1)), int(g.integers(256, wmax + 1))
        if g.uniform() < 0.5:
            h, w = w, h
        s = int(g.choice([2, 4, 8]))
        c = int(g.choice([1, 3]))
        specs.append(ImageSpec(h, w, c, radius_for(h, w), s, 1e-3, seed * 100003 + i))
    return specs


def image_for(spec: ImageSpec):
    I = photo_guide(spec.h, spec.w, spec.seed)
    return I, colour_input(I, spec.c, spec.seed + 1)


@dataclass
class Request:
    t_arrival: float
    spec: ImageSpec


_ASPECTS = [(1, 1), (4, 3), (3, 2), (16, 9)]


def request_mix(n: int, qps: float, seed: int = 7, mp_lo: float = 0.25, mp_hi: float = 24.0,
                s: int = 4) -> list[Request]:
    """Poisson arrivals at ``qps``; area log-uniform in [mp_lo, mp_hi] MP,
    aspect from {1:1, 4:3, 3:2, 16:9} in either orientation, C in {1,3} 50/50,
    r = round(0.01 max(H, W)), eps in {1e-2, 1e-3} 50/50."""
    g = _rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += g.exponential(1.0 / qps)
        area = math.exp(g.uniform(math.log(mp_lo), math.log(mp_hi))) * 1e6
        ah, aw = _ASPECTS[int(g.integers(0, len(_ASPECTS)))]
        if g.uniform() < 0.5:
            ah, aw = aw, ah
        h = max(1, int(round(math.sqrt(area * ah / aw))))
        w = max(1, int(round(area / h)))
        c = int(g.choice([1, 3]))
        eps = float(g.choice([1e-2, 1e-3]))
        reqs.append(Request(t, ImageSpec(h, w, c, radius_for(h, w), s, eps, seed * 100003 + i)))
    return reqs
