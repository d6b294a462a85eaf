"""Every tile shape of the window-sum kernels gives the oracle's result, and
the autotuner picks one of them and remembers it (GPU, through the C ABI)."""
import itertools
import os

import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


@pytest.mark.parametrize("h,w,c,r,s,sub", [(203, 347, 3, 9, 2, "bilinear"), (131, 257, 1, 7, 1, "nearest"),
                                         (90, 700, 2, 40, 4, "nearest")])
def test_every_tile_shape_matches_oracle(h, w, c, r, s, sub):
    import torch
    I = synth.photo_guide(h, w, seed=31)
    p = synth.colour_input(I, c, seed=32)
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), r, s, 1e-3, sub)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    ctx = gfp.Context(0)
    for cth, bth in itertools.product((8, 16, 24, 32, 48, 64), repeat=2):
        ctx.set_tiles(dI, dp, r, s, 1e-3, dict(coeff_th=cth, box_th=bth), sub)
        q = gfp.gf_fast(dI, dp, r, s, 1e-3, sub, ctx=ctx)
        torch.cuda.synchronize()
        e, where = gpuutil.max_err(gpuutil.stored_f64(q), exp)
        assert e <= 1e-5, (cth, bth, e, where)
    ctx.close()


@pytest.mark.parametrize("fusion", ["off", "on"])
def test_tuner_picks_a_candidate_and_persists(tmp_path, fusion):
    """The tuner times the coefficient candidates and the box-mean
    candidates, or, where the box means are fused into the output pass,
    that pass's candidates."""
    import torch
    I = synth.photo_guide(300, 400, seed=33)
    p = synth.colour_input(I, 3, seed=34)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    ctx = gfp.Context(0)
    ctx.set_fusion(fusion)
    best, rows = ctx.tune(dI, dp, 16, 4, 1e-3, reps=2)
    assert rows and all(ms > 0 for _, _, ms in rows)
    kernels = {k for k, _, _ in rows}
    assert kernels == ({"coeff", "box"} if fusion == "off" else {"coeff", "output"})
    # the chosen shapes are the fastest candidates of each kernel
    fastest = min((ms, t["coeff_th"]) for k, t, ms in rows if k == "coeff")[1]
    assert best["coeff_th"] == fastest
    fastest_box = min((ms, t["box_th"]) for k, t, ms in rows if k != "coeff")[1]
    assert best["box_th"] == fastest_box
    path = os.path.join(tmp_path, "tiles.json")
    ctx.save_tuning(path)
    ctx2 = gfp.Context(0)
    ctx2.set_fusion(fusion)
    ctx2.load_tuning(path)
    q1 = gfp.gf_fast(dI, dp, 16, 4, 1e-3, ctx=ctx)
    q2 = gfp.gf_fast(dI, dp, 16, 4, 1e-3, ctx=ctx2)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), 16, 4, 1e-3)
    assert gpuutil.max_err(gpuutil.stored_f64(q1), exp)[0] <= 1e-5
    ctx.close()
    ctx2.close()
