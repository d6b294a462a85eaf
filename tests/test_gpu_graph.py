"""A prepared batch (gf_batch_create / gf_batch_launch) captured into a HIP
graph and replayed: before every replay the inputs are rewritten and other
eager work runs; every replay must equal an eager gf_fast_batched on the
same inputs bit for bit, and the oracle within tolerance."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()

# (h, w, c, r, s, sub)
BATCH = [(300, 400, 3, 8, 4, "nearest"), (257, 129, 1, 5, 2, "bilinear"), (64, 64, 3, 3, 1, "nearest"),
         (511, 333, 1, 12, 8, "nearest"), (1, 500, 1, 4, 4, "nearest"), (220, 330, 5, 7, 2, "nearest")]
# r' = 60 does not fit the batched kernels' staged tiles: per-image kernels
PER_IMAGE = [(150, 170, 3, 60, 1, "nearest"), (90, 200, 1, 30, 2, "nearest")]


def content(spec, seed, dtype):
    h, w, c, *_ = spec
    I = synth.photo_guide(h, w, seed=seed)
    p = synth.colour_input(I, c, seed=seed + 1000)
    return gpuutil.to_device(I, dtype), gpuutil.to_device(p, dtype)


def run_graph_case(specs, dtype, schedule="phases", replays=3, borders=None):
    import torch
    print(f"graph case: {len(specs)} images, {dtype}, {schedule}", flush=True)
    Is, ps = map(list, zip(*[content(sp, 10 + k, dtype) for k, sp in enumerate(specs)]))
    borders = borders or ["clip"] * len(specs)
    prs = [gfp.params(r, s, 1e-3, sub, bd) for (_, _, _, r, s, sub), bd in zip(specs, borders)]
    bctx = gfp.Context(0)
    bctx.set_batch_cfg(schedule, 16)
    b = gfp.Batch(Is, ps, prs, ctx=bctx)
    # an eager launch of the prepared batch first (also loads its kernels)
    b.launch()
    ref = gfp.gf_fast_batched(Is, ps, prs, ctx=bctx)
    torch.cuda.synchronize()
    for k, (q, e) in enumerate(zip(b.qs, ref)):
        assert torch.equal(q, e), (k, specs[k])

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.launch()
    ctx = gfp.Context(0)
    for rep in range(replays):
        for k, sp in enumerate(specs):
            nI, npv = content(sp, 100 * (rep + 1) + k, dtype)
            Is[k].copy_(nI)
            ps[k].copy_(npv)
        for q in b.qs:
            q.fill_(float("nan"))  # a replay that writes nothing cannot pass
        # unrelated eager work through the library between replays
        h, w, c, r, s, sub = specs[0]
        gfp.gf_fast(Is[0], ps[0], r, s, 1e-3, sub, ctx=ctx, border=borders[0])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = gfp.gf_fast_batched(Is, ps, prs, ctx=bctx)
        torch.cuda.synchronize()
        for k, (sp, q, e) in enumerate(zip(specs, b.qs, ref)):
            assert torch.equal(q, e), (rep, k, sp)
        # one image per replay against the oracle
        k = rep % len(specs)
        h, w, c, r, s, sub = specs[k]
        exp = oracle.fast_guided_filter(gpuutil.stored_f64(Is[k]), gpuutil.stored_f64(ps[k]), r, s, 1e-3, sub,
                                        border=borders[k])
        got = gpuutil.stored_f64(b.qs[k])
        assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dtype, exp)), (rep, k, gpuutil.max_err(got, exp))
    del g
    ctx.close()
    b.close()
    bctx.close()


@pytest.mark.parametrize("schedule", ["phases", "queue"])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_graph_replays_batch(dtype, schedule):
    run_graph_case(BATCH, dtype, schedule)


def test_graph_replays_per_image_batch():
    run_graph_case(PER_IMAGE, "f32")


@pytest.mark.parametrize("schedule", ["phases", "queue"])
def test_graph_replays_padded_border_batch(schedule):
    """Batched kernels choose the border's tile code per task."""
    run_graph_case(BATCH, "f32", schedule,
                   borders=["reflect101", "replicate", "clip", "reflect101", "replicate", "clip"])


def test_graph_replays_area_batch():
    """Area subsampling: the batch runs image by image (area pass, then the
    per-image kernels), all captured in the graph."""
    specs = [(300, 400, 3, 8, 4, "area"), (257, 129, 1, 5, 2, "area"), (150, 151, 2, 6, 3, "nearest")]
    run_graph_case(specs, "f32", borders=["clip", "reflect101", "clip"])
