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


def coeff_shapes():
    for th in (4, 8, 16):
        yield dict(coeff_slide=1, coeff_th=th, coeff_tw=64, coeff_stage=1)
    for th, tw in itertools.product((16, 32), (32, 64)):
        yield dict(coeff_slide=0, coeff_th=th, coeff_tw=tw, coeff_stage=1)
    for th in (8, 16):
        yield dict(coeff_slide=0, coeff_th=th, coeff_tw=32, coeff_stage=0)


def box_shapes():
    for th in (4, 8, 16):
        yield dict(box_slide=1, box_th=th, box_stage=1)
    for th, st in itertools.product((8, 16, 32), (0, 1)):
        yield dict(box_slide=0, box_th=th, box_stage=st)


@pytest.mark.parametrize("h,w,c,r,s,sub", [(203, 347, 3, 9, 2, "bilinear"), (131, 257, 1, 7, 1, "nearest")])
def test_every_tile_shape_matches_oracle(h, w, c, r, s, sub):
    import torch
    I = synth.photo_guide(h, w, seed=31)
    p = synth.colour_input(I, c, seed=32)
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), r, s, 1e-3, sub)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    ctx = gfp.Context(0)
    default_box = dict(box_slide=1, box_th=8, box_stage=1)
    default_coeff = dict(coeff_slide=1, coeff_th=8, coeff_tw=64, coeff_stage=1)
    combos = [dict(**cs, **default_box) for cs in coeff_shapes()]
    combos += [dict(**default_coeff, **bs) for bs in box_shapes()]
    for t in combos:
        ctx.set_tiles(dI, dp, r, s, 1e-3, t, sub)
        q = gfp.gf_fast(dI, dp, r, s, 1e-3, sub, ctx=ctx)
        torch.cuda.synchronize()
        e, where = gpuutil.max_err(gpuutil.stored_f64(q), exp)
        assert e <= 1e-5, (t, e, where)
    ctx.close()


def test_tuner_picks_a_candidate_and_persists(tmp_path):
    import torch
    I = synth.photo_guide(300, 400, seed=33)
    p = synth.colour_input(I, 3, seed=34)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    ctx = gfp.Context(0)
    best, rows = ctx.tune(dI, dp, 16, 4, 1e-3, reps=2)
    assert rows and all(ms > 0 for _, _, ms in rows)
    kernels = {k for k, _, _ in rows}
    assert kernels == {"coeff", "box"}
    # the chosen coefficient shape is the fastest coefficient candidate
    fastest = min((ms, t) for k, t, ms in rows if k == "coeff")[1]
    assert all(best[f] == fastest[f] for f in ("coeff_slide", "coeff_th"))
    path = os.path.join(tmp_path, "tiles.json")
    ctx.save_tuning(path)
    ctx2 = gfp.Context(0)
    ctx2.load_tuning(path)
    q1 = gfp.gf_fast(dI, dp, 16, 4, 1e-3, ctx=ctx)
    q2 = gfp.gf_fast(dI, dp, 16, 4, 1e-3, ctx=ctx2)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    exp = oracle.fast_guided_filter(I.astype(np.float64), p.astype(np.float64), 16, 4, 1e-3)
    assert gpuutil.max_err(gpuutil.stored_f64(q1), exp)[0] <= 1e-5
    ctx.close()
    ctx2.close()
