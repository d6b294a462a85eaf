"""Colour (three-channel) guidance on the GPU through the C ABI: the plain
and fast filters against the FP64 oracle, element by element.

Tolerance as for the gray guide: max|q_gpu - q_oracle| <= 1e-5 with FP32
storage; with 16-bit storage 2e-3 (bf16 outputs with |q| >= 1: half a bf16
ulp + 1e-4) and half an ulp + 1e-5 per element, and the 16-bit q equals the
FP32 path's q rounded once.  The coefficients are solved in FP64 and rounded once to FP32;
q = mean_a.I + mean_b is formed in FP32 with one rounding per term."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def check(h, w, c, r, s, sub, border, dt, eps=1e-3, seed=0, coeff_th=None):
    """coeff_th: pin the coefficient tile height (16 rows where they fit by
    default; 8 when pinned to 8)."""
    import torch
    print(f"colour case: {h}x{w}x{c} r={r} s={s} {sub} {border} {dt} tiles {coeff_th}", flush=True)
    I = synth.colour_guide(h, w, seed=300 + seed + h)
    p = synth.colour_input(I.mean(axis=0, dtype=np.float32), c, seed=400 + seed + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    ctx = gfp.Context(0)
    if coeff_th is not None:
        ctx.set_tiles(dI, dp, r, s, eps, dict(coeff_th=coeff_th, box_th=24), sub)
    q = (gfp.gf_plain(dI, dp, r, eps, border=border, ctx=ctx) if s == 1 else
         gfp.gf_fast(dI, dp, r, s, eps, sub, border=border, ctx=ctx))
    torch.cuda.synchronize()
    exp = oracle.fast_guided_filter_color(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, s, eps, sub, border)
    got = gpuutil.stored_f64(q)
    assert got.shape == exp.shape
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), gpuutil.max_err(got, exp)
    if dt != "f32":  # the 16-bit q is the FP32 path's q rounded once
        dI32, dp32 = dI.float(), dp.float()
        if coeff_th is not None:  # tiles are pinned per storage type: same tiles, same sums
            ctx.set_tiles(dI32, dp32, r, s, eps, dict(coeff_th=coeff_th, box_th=24), sub)
        q32 = (gfp.gf_plain(dI32, dp32, r, eps, border=border, ctx=ctx) if s == 1 else
               gfp.gf_fast(dI32, dp32, r, s, eps, sub, border=border, ctx=ctx))
        torch.cuda.synchronize()
        gpuutil.split_16bit(q, q32, exp)
    ctx.close()
    return dI, dp, q


# (h, w, c, r, s, sub, border, dtype)
CASES = [
    (300, 400, 3, 16, 4, "nearest", "clip", "f32"),
    (257, 129, 1, 8, 2, "bilinear", "clip", "f32"),
    (150, 151, 2, 6, 1, "nearest", "clip", "f32"),          # Algorithm 1 with a colour guide
    (201, 199, 1, 10, 5, "nearest", "clip", "f32"),         # ratio without compile-time taps
    (511, 333, 3, 24, 8, "nearest", "reflect101", "f32"),
    (150, 170, 1, 12, 3, "area", "replicate", "f32"),
    (33, 47, 1, 40, 4, "nearest", "reflect101", "f32"),     # r' = 10 > 9 rows
    (1, 500, 1, 4, 4, "nearest", "clip", "f32"),            # one low-res row
    (500, 3, 2, 12, 4, "bilinear", "clip", "f32"),          # one low-res column
    (120, 100, 5, 20, 1, "nearest", "replicate", "f32"),    # 5 channels, r = 20 at full resolution
    (400, 600, 3, 16, 4, "nearest", "clip", "f16"),
    (222, 350, 3, 12, 4, "bilinear", "clip", "bf16"),
    (240, 320, 3, 16, 4, "area", "clip", "f16"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_color_matches_oracle(case):
    check(*case)


@pytest.mark.parametrize("th", [8, 16])
@pytest.mark.parametrize("case", [(203, 347, 3, 9, 2, "bilinear", "clip", "f32"),
                                  (150, 151, 2, 16, 1, "nearest", "reflect101", "f32"),
                                  (300, 400, 3, 16, 4, "area", "clip", "f16"),
                                  (77, 520, 1, 36, 3, "nearest", "replicate", "f32")],
                         ids=lambda c: "x".join(map(str, c)))
def test_color_tile_heights(case, th):
    """Both coefficient tile heights of the colour guide: 16 rows (the
    default where they fit) and 8 (pinned), ragged tiles included."""
    check(*case, coeff_th=th)


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_color_12mp(eps):
    """4000x3000 RGB guide, RGB input, r = 16, s = 4, fp32 (every element)."""
    import torch
    I, p = synth.workload_12mp_colour()
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    q = gfp.gf_fast(dI, dp, 16, 4, eps)
    torch.cuda.synchronize()
    exp = oracle.fast_guided_filter_color(I.astype(np.float64), p.astype(np.float64), 16, 4, eps)
    err = float(np.max(np.abs(q.double().cpu().numpy() - exp)))
    assert err <= 1e-5, err


def test_color_equal_planes_is_gray():
    """A guide of three equal planes G gives the gray filter of G at eps/3."""
    import torch
    G = synth.photo_guide(260, 310, seed=9)
    p = synth.colour_input(G, 2, seed=10)
    dG, dp = gpuutil.to_device(G), gpuutil.to_device(p)
    dI = torch.stack([dG, dG, dG]).contiguous()
    qc = gfp.gf_fast(dI, dp, 12, 4, 3e-3)
    qg = gfp.gf_fast(dG, dp, 12, 4, 1e-3)
    torch.cuda.synchronize()
    assert float((qc.double() - qg.double()).abs().max()) <= 2e-5


def test_color_batched_runs_per_image():
    """A batch holding colour-guided images runs image by image: the same
    bits as gf_fast for every image, gray ones included."""
    import torch
    specs = [(3, 200, 260, 2, 8, 4), (1, 150, 151, 1, 6, 2), (3, 90, 70, 3, 5, 1)]
    Is, ps, prs = [], [], []
    for k, (gc, h, w, c, r, s) in enumerate(specs):
        I = synth.colour_guide(h, w, seed=20 + k) if gc == 3 else synth.photo_guide(h, w, seed=20 + k)
        Is.append(gpuutil.to_device(I))
        ps.append(gpuutil.to_device(synth.colour_input(I if gc == 1 else I.mean(axis=0), c, seed=30 + k)))
        prs.append(gfp.params(r, s, 1e-3))
    qs = gfp.gf_fast_batched(Is, ps, prs)
    torch.cuda.synchronize()
    for k, (gc, h, w, c, r, s) in enumerate(specs):
        solo = gfp.gf_fast(Is[k], ps[k], r, s, 1e-3)
        torch.cuda.synchronize()
        assert torch.equal(qs[k], solo), specs[k]


@pytest.mark.parametrize("s,sub,border,dt", [(4, "nearest", "clip", "f32"), (2, "bilinear", "reflect101", "f32"),
                                              (3, "area", "replicate", "f32"), (4, "nearest", "clip", "f16")])
def test_color_joint_upsample(s, sub, border, dt):
    """A low-res RGB input guided by a full-res RGB guide, against the oracle."""
    import torch
    h, w, c, r = 301, 405, 3, 16
    I = synth.colour_guide(h, w, seed=41)
    g = np.random.Generator(np.random.PCG64(42))
    p_lo = g.uniform(0, 1, size=(c, -(-h // s), -(-w // s))).astype(np.float32)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p_lo, dt)
    q = gfp.gf_joint_upsample(dI, dp, r, s, 1e-3, sub, border=border)
    torch.cuda.synchronize()
    exp = oracle.joint_upsample_color(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, s, 1e-3, sub, border)
    got = gpuutil.stored_f64(q)
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), gpuutil.max_err(got, exp)


@pytest.mark.parametrize("s,dt", [(4, "f32"), (1, "f32"), (8, "bf16"), (4, "f16")])
def test_color_detail_enhance(s, dt):
    """e = q + 5 (p - q) with q the colour-guided filter; tolerance as for
    the gray guide's detail test (q kept in FP32, e rounded once)."""
    import torch
    h, w, c, gain = 250, 330, 3, 5.0
    I = synth.colour_guide(h, w, seed=51)
    p = synth.colour_input(I.mean(axis=0, dtype=np.float32), c, seed=52)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    e = gfp.gf_detail_enhance(dI, dp, 16, s, 1e-2, gain)
    torch.cuda.synchronize()
    I64, p64 = gpuutil.stored_f64(dI), gpuutil.stored_f64(dp)
    q = oracle.fast_guided_filter_color(I64, p64, 16, s, 1e-2)
    exp = oracle.detail_enhance(p64, q, gain)
    got = gpuutil.stored_f64(e)
    assert np.all(np.abs(got - exp) <= gpuutil.detail_tolerance(dt, exp, p64, q, gain)), gpuutil.max_err(got, exp)


def test_color_tuner_refused():
    I = gpuutil.to_device(synth.colour_guide(64, 64, seed=1))
    p = gpuutil.to_device(synth.photo_guide(64, 64, seed=2))[None]
    with gfp.Context(0) as ctx:
        with pytest.raises(gfp.GfError) as ei:
            ctx.tune(I, p, 8, 4, 1e-2)
        assert ei.value.status == gfp.GF_ENOTSUP


def test_color_served_like_solo():
    """gf_submit admits a colour-guided request alone (per-image kernels):
    the result equals gf_fast, also with gray requests queued around it
    (those equal gf_fast with the batched kernels' tiles)."""
    import torch
    Ic = gpuutil.to_device(synth.colour_guide(180, 240, seed=61))
    Ig = gpuutil.to_device(synth.photo_guide(180, 240, seed=62))
    p = gpuutil.to_device(synth.colour_input(synth.photo_guide(180, 240, seed=62), 3, seed=63))
    with gfp.Context(0, arena_bytes=1 << 27, max_inflight=8) as ctx:
        guides = [Ig, Ic, Ig, Ic]
        qs = [torch.empty_like(p) for _ in guides]
        tickets = [ctx.gf_submit(I, p, q, 8, 4, 1e-2) for I, q in zip(guides, qs)]
        for t in tickets:
            st, _ = ctx.gf_poll(t, 10000)
            assert st == gfp.GF_OK
        pin = gfp.Context(0)
        pin.set_tiles(Ig, p, 8, 4, 1e-2, gpuutil.batch_tiles("phases", 24))
        for I, q in zip(guides, qs):
            solo = gfp.gf_fast(I, p, 8, 4, 1e-2, ctx=pin if I is Ig else None)
            torch.cuda.synchronize()
            assert torch.equal(q, solo)
        pin.close()
