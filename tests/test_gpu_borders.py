"""Padded borders (replicate, reflect-101) and area subsampling on the GPU,
through the C ABI, against the FP64 oracle; and their batched and served
forms against the per-image entry point.

Tolerances as for the clip-normalised filter (max|q_gpu - q_oracle| <= 1e-5
with FP32 storage; with 16-bit storage 2e-3, bf16 outputs with |q| >= 1:
half a bf16 ulp + 1e-4, and half an ulp + 1e-5 per element; the 16-bit q is
the FP32 path's q rounded once).  Area subsampling rounds the block means of I and p
once to FP32 (the oracle keeps them in FP64); at eps >= 1e-3 that moves q by
far less than the tolerance."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def check(h, w, c, r, s, sub, border, dt, eps=1e-3, seed=0, plain=False):
    import torch
    print(f"borders case: {h}x{w}x{c} r={r} s={s} {sub} {border} {dt}", flush=True)
    I = synth.photo_guide(h, w, seed=900 + seed + h)
    p = synth.colour_input(I, c, seed=950 + seed + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    q = gfp.gf_plain(dI, dp, r, eps, border=border) if plain else gfp.gf_fast(dI, dp, r, s, eps, sub, border=border)
    torch.cuda.synchronize()
    Is, ps = gpuutil.stored_f64(dI), gpuutil.stored_f64(dp)
    if plain:
        exp = oracle.guided_filter(Is, ps, r, eps, border=border)
    else:
        exp = oracle.fast_guided_filter(Is, ps, r, s, eps, sub, border=border)
    got = gpuutil.stored_f64(q)
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), gpuutil.max_err(got, exp)
    if dt != "f32":  # the 16-bit q is the FP32 path's q rounded once
        dI32, dp32 = dI.float(), dp.float()
        q32 = (gfp.gf_plain(dI32, dp32, r, eps, border=border) if plain else
               gfp.gf_fast(dI32, dp32, r, s, eps, sub, border=border))
        torch.cuda.synchronize()
        gpuutil.split_16bit(q, q32, exp)
    return dI, dp, q


# (h, w, c, r, s, sub, border, dtype)
BORDER_CASES = [
    (300, 400, 3, 16, 4, "nearest", "replicate", "f32"),
    (300, 400, 3, 16, 4, "nearest", "reflect101", "f32"),
    (257, 129, 1, 8, 2, "bilinear", "reflect101", "f32"),
    (257, 129, 1, 8, 2, "bilinear", "replicate", "f32"),
    (150, 151, 2, 6, 1, "nearest", "reflect101", "f32"),     # Algorithm 1 (s = 1)
    (33, 47, 1, 40, 4, "nearest", "reflect101", "f32"),     # r' = 10 > 9 rows: repeated reflection
    (1, 500, 1, 4, 4, "nearest", "reflect101", "f32"),      # one low-res row
    (500, 3, 2, 12, 4, "bilinear", "replicate", "f32"),     # one low-res column
    (511, 333, 3, 24, 8, "nearest", "reflect101", "f32"),
    (400, 600, 3, 16, 4, "nearest", "replicate", "f16"),
    (222, 350, 3, 12, 4, "bilinear", "reflect101", "bf16"),
]


@pytest.mark.parametrize("case", BORDER_CASES, ids=lambda c: "x".join(map(str, c)))
def test_border_matches_oracle(case):
    check(*case)


@pytest.mark.parametrize("border", ["replicate", "reflect101"])
def test_border_plain_unstaged_radius(border):
    """r = 60 at s = 1: the coefficient tiles are too large to stage in LDS
    and read their samples through the caches."""
    check(150, 170, 1, 60, 1, "nearest", border, "f32", plain=True)


AREA_CASES = [
    (300, 400, 3, 16, 4, "area", "clip", "f32"),
    (257, 131, 1, 8, 3, "area", "clip", "f32"),     # odd ratio, ragged blocks on both axes
    (201, 199, 1, 10, 5, "area", "clip", "f32"),
    (511, 333, 2, 24, 8, "area", "replicate", "f32"),
    (150, 151, 1, 6, 2, "area", "reflect101", "f32"),
    (7, 1000, 3, 8, 8, "area", "clip", "f32"),      # one block row, shorter than s
    (600, 800, 3, 16, 4, "area", "clip", "f16"),
    (420, 380, 3, 12, 4, "area", "reflect101", "bf16"),
]


@pytest.mark.parametrize("case", AREA_CASES, ids=lambda c: "x".join(map(str, c)))
def test_area_matches_oracle(case):
    check(*case)


def test_area_s1_is_plain():
    """At s = 1 the area mean of a pixel is the pixel: same bits as nearest."""
    import torch
    I = synth.photo_guide(120, 130, seed=5)
    p = synth.colour_input(I, 2, seed=6)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    qa = gfp.gf_fast(dI, dp, 6, 1, 1e-3, "area")
    qn = gfp.gf_fast(dI, dp, 6, 1, 1e-3, "nearest")
    torch.cuda.synchronize()
    assert torch.equal(qa, qn)


def test_area_12mp():
    """4000x3000 RGB, r = 16, s = 4, area subsampling, fp32, against the oracle."""
    import torch
    h, w, c = 3000, 4000, 3
    I, p = synth.workload_12mp(h, w, c)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    q = gfp.gf_fast(dI, dp, 16, 4, 1e-2, "area")
    torch.cuda.synchronize()
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), 16, 4, 1e-2, "area")
    err = float(np.max(np.abs(q.double().cpu().numpy() - exp)))
    assert err <= 1e-5, err


@pytest.mark.parametrize("sub,border", [("area", "clip"), ("nearest", "reflect101"), ("area", "replicate")])
def test_joint_upsample_border_area(sub, border):
    import torch
    h, w, c, r, s = 301, 405, 3, 16, 4
    I = synth.photo_guide(h, w, seed=21)
    g = np.random.Generator(np.random.PCG64(22))
    p_lo = g.uniform(0, 1, size=(c, -(-h // s), -(-w // s))).astype(np.float32)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p_lo)
    q = gfp.gf_joint_upsample(dI, dp, r, s, 1e-3, sub, border=border)
    torch.cuda.synchronize()
    exp = oracle.joint_upsample(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, s, 1e-3, sub, border=border)
    got = gpuutil.stored_f64(q)
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance("f32", exp)), gpuutil.max_err(got, exp)


def test_detail_enhance_area_reflect():
    """The detail epilogue over an area-subsampled, reflect-101 filter."""
    import torch
    h, w, c = 240, 330, 3
    I = synth.photo_guide(h, w, seed=31)
    p = synth.colour_input(I, c, seed=32)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    e = gfp.gf_detail_enhance(dI, dp, 16, 4, 1e-2, 5.0, "area", border="reflect101")
    q = gfp.gf_fast(dI, dp, 16, 4, 1e-2, "area", border="reflect101")
    torch.cuda.synchronize()
    exp_q = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), 16, 4, 1e-2, "area",
                                      border="reflect101")
    exp = oracle.detail_enhance(p.astype(np.float64), exp_q, 5.0)
    assert float(np.max(np.abs(q.double().cpu().numpy() - exp_q))) <= 1e-5
    tol = gpuutil.detail_tolerance("f32", exp, p.astype(np.float64), exp_q, 5.0)
    assert np.all(np.abs(e.double().cpu().numpy() - exp) <= tol)


# a batch mixing every border (the batched kernels read the convention per image)
MIXED = [(300, 400, 3, 8, 4, "nearest", "replicate"), (257, 129, 1, 5, 2, "bilinear", "reflect101"),
         (64, 64, 3, 3, 1, "nearest", "clip"), (33, 47, 1, 40, 4, "nearest", "reflect101"),
         (1, 500, 1, 4, 4, "nearest", "replicate"), (220, 330, 2, 7, 8, "nearest", "reflect101")]


def batch_vs_solo(specs, dtype, schedule, th=16):
    """Batched (tile height th) against gf_fast with the same tile shapes
    (th = 0: a batch that runs image by image, with the built-in shapes)."""
    import torch
    Is, ps, prs = [], [], []
    for k, (h, w, c, r, s, sub, border) in enumerate(specs):
        I = synth.photo_guide(h, w, seed=40 + k)
        Is.append(gpuutil.to_device(I, dtype))
        ps.append(gpuutil.to_device(synth.colour_input(I, c, seed=60 + k), dtype))
        prs.append(gfp.params(r, s, 1e-3, sub, border))
    ctx = gfp.Context(0)
    ctx.set_batch_cfg(schedule, th)
    qs = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
    torch.cuda.synchronize()
    for k, (h, w, c, r, s, sub, border) in enumerate(specs):
        if th:
            ctx.set_tiles(Is[k], ps[k], r, s, 1e-3, gpuutil.batch_tiles(schedule, th), sub)
        solo = gfp.gf_fast(Is[k], ps[k], r, s, 1e-3, sub, ctx=ctx, border=border)
        torch.cuda.synchronize()
        assert torch.equal(qs[k], solo), (k, specs[k])
    ctx.close()
    return Is, ps, qs


@pytest.mark.parametrize("schedule", ["phases", "queue"])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_batched_borders_equal_solo(dtype, schedule):
    Is, ps, qs = batch_vs_solo(MIXED, dtype, schedule)
    k = 1  # and one image against the oracle
    h, w, c, r, s, sub, border = MIXED[k]
    exp = oracle.fast_guided_filter(gpuutil.stored_f64(Is[k]), gpuutil.stored_f64(ps[k]), r, s, 1e-3, sub,
                                    border=border)
    got = gpuutil.stored_f64(qs[k])
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dtype, exp)), gpuutil.max_err(got, exp)


def test_batched_with_area_runs_per_image():
    """A batch holding an area-subsampled image runs image by image: same
    bits as gf_fast for every image."""
    batch_vs_solo(MIXED[:2] + [(150, 151, 1, 6, 4, "area", "clip"), (70, 90, 3, 8, 2, "area", "reflect101")],
                  "f32", "phases", th=0)


def test_served_border_and_area():
    """gf_submit runs a padded-border request (batched kernels) and an
    area-subsampled one (per-image kernels, admitted alone) like gf_fast,
    interleaved with plain requests."""
    import torch
    I = synth.photo_guide(200, 260, seed=71)
    p = synth.colour_input(I, 3, seed=72)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    kinds = [("nearest", "reflect101"), ("area", "clip"), ("nearest", "clip"), ("area", "replicate"),
             ("bilinear", "replicate")]
    with gfp.Context(0, arena_bytes=1 << 28, max_inflight=8) as ctx:
        qs, tickets = [], []
        for sub, border in kinds:
            qs.append(torch.empty_like(dp))
            tickets.append(ctx.gf_submit(dI, dp, qs[-1], 12, 4, 1e-3, sub, border))
        for t in tickets:
            st, _ = ctx.gf_poll(t, 10000)
            assert st == gfp.GF_OK
        # the batched requests against gf_fast with the batched kernels'
        # tiles; the area ones ran the per-image kernels with their own
        pin = gfp.Context(0)
        pin.set_tiles(dI, dp, 12, 4, 1e-3, gpuutil.batch_tiles("phases", 24))
        for q, (sub, border) in zip(qs, kinds):
            solo = gfp.gf_fast(dI, dp, 12, 4, 1e-3, sub, border=border, ctx=None if sub == "area" else pin)
            torch.cuda.synchronize()
            assert torch.equal(q, solo), (sub, border)
        pin.close()
