"""Persistent batched launch (gf_fast_batched): every image of a mixed batch
equals the oracle within tolerance and equals a solo gf_fast of that image
run with the same tile shapes (GPU, through the C ABI)."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()

# (h, w, c, r, s, sub)
MIX = [(300, 400, 3, 8, 4, "nearest"), (257, 129, 1, 5, 2, "bilinear"), (64, 64, 3, 3, 1, "nearest"),
       (511, 333, 1, 12, 8, "nearest"), (97, 1003, 3, 6, 4, "bilinear"), (1, 500, 1, 4, 4, "nearest"),
       (400, 1, 3, 4, 2, "nearest"), (150, 151, 2, 9, 3, "bilinear"), (600, 800, 3, 16, 4, "nearest"),
       (33, 47, 1, 0, 4, "nearest"), (700, 300, 1, 20, 4, "bilinear"), (220, 330, 5, 7, 2, "nearest")]


def make(spec, k, dtype):
    h, w, c, r, s, sub = spec
    I = synth.photo_guide(h, w, seed=100 + k)
    p = synth.colour_input(I, c, seed=200 + k)
    return gpuutil.to_device(I, dtype), gpuutil.to_device(p, dtype)


@pytest.mark.parametrize("schedule,th", [("phases", 16), ("queue", 16), ("phases", 8), ("queue", 24), ("phases", 32),
                                         ("phases", 48)])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_mixed_batch_matches_oracle_and_solo(dtype, schedule, th):
    import torch
    print(f"mixed batch {dtype} {schedule} th={th}", flush=True)
    imgs = [make(sp, k, dtype) for k, sp in enumerate(MIX)]
    Is = [a for a, _ in imgs]
    ps = [b for _, b in imgs]
    prs = [gfp.params(r, s, 1e-3, sub) for (_, _, _, r, s, sub) in MIX]
    ctx = gfp.Context(0)
    ctx.set_batch_cfg(schedule, th)
    qs = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
    torch.cuda.synchronize()
    for k, ((h, w, c, r, s, sub), dI, dp, q) in enumerate(zip(MIX, Is, ps, qs)):
        exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp if c > 1 else dp),
                                        r, s, 1e-3, sub)
        got = gpuutil.stored_f64(q)
        tol = gpuutil.tolerance(dtype, exp)
        assert np.all(np.abs(got - exp) <= tol), (k, MIX[k], gpuutil.max_err(got, exp))
        # the same image alone, with the tile shapes the batched kernel uses
        ctx.set_tiles(dI, dp, r, s, 1e-3, gpuutil.batch_tiles(schedule, th), sub)
        solo = gfp.gf_fast(dI, dp, r, s, 1e-3, sub, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(solo, q), (k, MIX[k], float((solo.float() - q.float()).abs().max()))
    ctx.close()


def test_batch_from_generator_fp16():
    """A batch drawn like the 256-image workload (smaller sizes to keep the
    oracle quick): mixed sizes and aspect ratios, r = round(0.01 max(H, W)),
    s in {2, 4, 8}, C in {1, 3}, eps = 1e-3, fp16 storage."""
    import torch
    specs = synth.batch_specs(24, seed=6, hmax=512, wmax=640)
    Is, ps, prs = [], [], []
    for sp in specs:
        I, p = synth.image_for(sp)
        Is.append(gpuutil.to_device(I, "f16"))
        ps.append(gpuutil.to_device(p, "f16"))
        prs.append(gfp.params(sp.r, sp.s, sp.eps))
    qs = gfp.gf_fast_batched(Is, ps, prs)
    torch.cuda.synchronize()
    for sp, dI, dp, q in zip(specs, Is, ps, qs):
        exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), sp.r, sp.s, sp.eps)
        got = gpuutil.stored_f64(q)
        assert np.all(np.abs(got - exp) <= gpuutil.tolerance("f16", exp)), (sp, gpuutil.max_err(got, exp))


def test_batch_repeated_launches_are_identical():
    import torch
    imgs = [make(sp, k, "f32") for k, sp in enumerate(MIX[:6])]
    Is, ps = [a for a, _ in imgs], [b for _, b in imgs]
    prs = [gfp.params(r, s, 1e-3, sub) for (_, _, _, r, s, sub) in MIX[:6]]
    ctx = gfp.Context(0)
    q1 = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
    q2 = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
    torch.cuda.synchronize()
    for a, b in zip(q1, q2):
        assert torch.equal(a, b)
    ctx.close()


def test_batch_rejects_bad_input():
    import torch
    (I1, p1), (I2, p2) = make(MIX[0], 0, "f32"), make(MIX[1], 1, "f16")
    with pytest.raises(gfp.GfError) as e:
        gfp.gf_fast_batched([I1, I2], [p1, p2], [gfp.params(8, 4, 1e-3)] * 2)
    assert e.value.status == gfp.GF_EINVAL
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(gfp.GfError) as e:
        gfp.gf_fast_batched([I1], [p1], [gfp.params(8, 4, 1e-3)], workspace=ws)
    assert e.value.status == gfp.GF_ENOMEM


@pytest.mark.parametrize("schedule", ["phases", "queue"])
def test_batch_tuner_picks_a_measured_configuration(schedule):
    """The tuner times the tile heights of the phase schedule, or of the
    queue schedule when the context is set to it."""
    import torch
    imgs = [make(sp, k, "f16") for k, sp in enumerate(MIX)]
    Is, ps = [a for a, _ in imgs], [b for _, b in imgs]
    prs = [gfp.params(r, s, 1e-3, sub) for (_, _, _, r, s, sub) in MIX]
    ctx = gfp.Context(0)
    ctx.set_batch_cfg(schedule)
    best, rows = ctx.tune_batched(Is, ps, prs, reps=2)
    assert rows and best in [c for c, _ in rows]
    assert min(rows, key=lambda x: x[1])[0] == best
    assert {c["schedule"] for c, _ in rows} == {schedule}
    assert len(rows) >= 3
    # the context now launches batches with the chosen configuration: same bits as solo runs
    qs = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
    torch.cuda.synchronize()
    for (h, w, c, r, s, sub), dI, dp, q in zip(MIX, Is, ps, qs):
        ctx.set_tiles(dI, dp, r, s, 1e-3, gpuutil.batch_tiles(best["schedule"], best["tile_h"]), sub)
        solo = gfp.gf_fast(dI, dp, r, s, 1e-3, sub, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(solo, q), (h, w, c, r, s, sub, best)
    ctx.close()
