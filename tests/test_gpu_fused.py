"""Box means fused into the output pass (Algorithm 2 steps 5-7 in one launch)
against the three-pass path (separate box-mean pass) on the GPU through the
C ABI.

The fused pass sums the box means of a and b in the same runs and order as
the box-mean pass with the same tiles, so q must be the same bit for bit:
every case runs the same call on a context with fusion on and on one with
fusion off and compares with torch.equal, and checks the fused q against the
FP64 oracle (max|q - q_oracle| <= 1e-5 for FP32 storage; the 16-bit bounds
of gpuutil.tolerance).  The kernel counts show which path ran."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


FUSED_TILES = dict(coeff_th=16, box_th=8)


def run_pair(dI, dp, r, s, eps, sub, border, tiles=FUSED_TILES, call="fast", gain=5.0):
    """q with fusion on and off (the same tiles pinned on both contexts), and
    the kernel counts of the fused run."""
    import torch
    out = []
    counts = None
    for fuse in (True, False):
        ctx = gfp.Context(0)
        ctx.set_fusion("on" if fuse else "off")
        if tiles is not None:
            ctx.set_tiles(dI, dp, r, s, eps, tiles, sub)
        ctx.profile(True)
        if call == "fast":
            q = gfp.gf_fast(dI, dp, r, s, eps, sub, ctx=ctx, border=border)
        elif call == "detail":
            q = gfp.gf_detail_enhance(dI, dp, r, s, eps, gain, sub, ctx=ctx, border=border)
        else:  # joint upsampling: dp is the low-res input
            q = gfp.gf_joint_upsample(dI, dp, r, s, eps, sub, ctx=ctx, border=border)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        if fuse:
            counts = {k: v[1] for k, v in prof.items()}
        ctx.close()
        out.append(q)
    return out[0], out[1], counts


# (h, w, c, r, s, sub, border, dtype)
CASES = [
    (300, 400, 3, 16, 4, "nearest", "clip", "f32"),
    (301, 257, 1, 8, 2, "bilinear", "clip", "f32"),
    (257, 519, 2, 24, 8, "nearest", "clip", "f32"),
    (1, 700, 1, 8, 4, "nearest", "clip", "f32"),          # one full-res row
    (700, 1, 1, 8, 4, "nearest", "clip", "f32"),          # one full-res column
    (1, 1, 1, 3, 2, "nearest", "clip", "f32"),
    (33, 45, 3, 0, 4, "nearest", "clip", "f32"),          # r = 0: one-pixel windows
    (65, 97, 1, 40, 4, "nearest", "clip", "f32"),         # r' = 10 > the low-res map
    (200, 300, 3, 16, 4, "nearest", "replicate", "f32"),
    (211, 173, 2, 12, 2, "bilinear", "reflect101", "f32"),
    (90, 130, 1, 60, 8, "nearest", "reflect101", "f32"),  # windows wider than the map
    (150, 170, 3, 12, 4, "area", "clip", "f32"),
    (129, 255, 5, 10, 4, "nearest", "clip", "f32"),       # five channels
    (400, 600, 3, 32, 8, "nearest", "clip", "f16"),
    (400, 600, 3, 16, 4, "nearest", "clip", "bf16"),
    (333, 517, 3, 12, 2, "bilinear", "clip", "f16"),
    (222, 350, 1, 8, 4, "area", "reflect101", "bf16"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_fused_equals_three_pass(case):
    h, w, c, r, s, sub, border, dt = case
    print(f"fused case: {h}x{w}x{c} r={r} s={s} {sub} {border} {dt}", flush=True)
    I = synth.photo_guide(h, w, seed=1000 + h)
    p = synth.colour_input(I, c, seed=1100 + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    qf, qu, counts = run_pair(dI, dp, r, s, 1e-3, sub, border)
    assert counts["box"] == 0 and counts["output"] == 1, counts  # the fused pass ran
    assert qf.shape == qu.shape
    assert bool((qf == qu).all()), f"{int((qf != qu).sum())} elements differ from the three-pass q"
    exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, s, 1e-3, sub,
                                    border=border)
    got = gpuutil.stored_f64(qf)
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), gpuutil.max_err(got, exp)


@pytest.mark.parametrize("box_th", [8, 16, 24, 32, 48, 64])
@pytest.mark.parametrize("case", [(517, 389, 3, 12, 4, "nearest", "clip", "f32"),
                                  (300, 700, 2, 20, 2, "nearest", "reflect101", "f16"),
                                  (260, 900, 1, 24, 8, "bilinear", "clip", "bf16")],
                         ids=lambda c: "x".join(map(str, c)))
def test_fused_every_box_tile_height(case, box_th):
    """Every box tile height (column runs of box_th / 4 rows) gives the bits
    of the box-mean pass with that height (at s = 2 and r' = 10 the taller
    heights need more LDS than the fused pass takes and run three passes)."""
    h, w, c, r, s, sub, border, dt = case
    print(f"fused tiles case: {h}x{w}x{c} r={r} s={s} {sub} {border} {dt} box_th={box_th}", flush=True)
    I = synth.photo_guide(h, w, seed=1200 + h)
    p = synth.colour_input(I, c, seed=1300 + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    qf, qu, counts = run_pair(dI, dp, r, s, 1e-3, sub, border, tiles=dict(coeff_th=16, box_th=box_th))
    fused = counts["box"] == 0
    assert fused or (s == 2 and box_th >= 32), counts
    assert bool((qf == qu).all()), f"box_th {box_th}: {int((qf != qu).sum())} elements differ"


def test_fused_detail_and_joint():
    """The detail-enhancement epilogue and joint upsampling take the fused
    pass too, with the same bits."""
    import torch
    I = synth.photo_guide(411, 623, seed=77)
    p = synth.colour_input(I, 3, seed=78)
    for dt in ("f32", "f16"):
        print(f"fused detail/joint {dt}", flush=True)
        dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
        ef, eu, counts = run_pair(dI, dp, 16, 4, 1e-2, "nearest", "clip", call="detail")
        assert counts["box"] == 0 and bool((ef == eu).all())
        plow = dp[:, 2::4, 2::4].contiguous()
        jf, ju, counts = run_pair(dI, plow, 16, 4, 1e-3, "nearest", "clip", call="joint")
        assert counts["box"] == 0 and bool((jf == ju).all())
        ctx = gfp.Context(0)  # joint of the nearest subsample = fast, with the same tiles
        ctx.set_tiles(dI, dp, 16, 4, 1e-3, FUSED_TILES)
        assert torch.equal(jf, gfp.gf_fast(dI, dp, 16, 4, 1e-3, ctx=ctx))
        ctx.close()


def test_unfused_where_it_does_not_apply():
    """s = 1, s = 3 and a colour guide keep the separate box-mean pass."""
    I = synth.photo_guide(150, 200, seed=5)
    p = synth.colour_input(I, 2, seed=6)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    for s in (1, 3):
        qf, qu, counts = run_pair(dI, dp, 6, s, 1e-3, "nearest", "clip")
        assert counts["box"] == 1 and bool((qf == qu).all()), (s, counts)
    G = synth.colour_guide(150, 200, seed=7)
    dG = gpuutil.to_device(G)
    qf, qu, counts = run_pair(dG, dp, 8, 4, 1e-3, "nearest", "clip")
    assert counts["box"] == 1 and bool((qf == qu).all()), counts


def test_fused_12mp_headline():
    """The 4000x3000 RGB workload at r = 16, s = 4: fused equals three-pass
    and the oracle (every element)."""
    I, p = synth.workload_12mp()
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    qf, qu, counts = run_pair(dI, dp, 16, 4, 1e-3, "nearest", "clip")
    assert counts["box"] == 0 and bool((qf == qu).all())
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), 16, 4, 1e-3)
    assert float(np.max(np.abs(gpuutil.stored_f64(qf) - exp))) <= 1e-5
