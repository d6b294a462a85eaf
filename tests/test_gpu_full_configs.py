"""The batched and served workloads at their full sizes and in the launch
configurations the benchmark times, every output of every image against the
oracle (GPU, through the C ABI):

* the 256-image batch (H up to 1536, W up to 2048, either orientation,
  s in {2, 4, 8}, C in {1, 3}, r = round(0.01 max(H, W)), fp16) under both
  schedules at 24-row coefficient tiles, the height the batch autotuner
  picks;
* requests of 0.25-24 MP (log-uniform area, C in {1, 3}, s = 4, fp16)
  through gf_submit / gf_poll with the benchmark's 4 GiB arena, plus one
  request at the 24 MP maximum.

Pixel values are seeded uniform noise made on the GPU, as the benchmark
fills these workloads."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def noise_images(torch, specs, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    Is, ps = [], []
    for sp in specs:
        Is.append(torch.rand((sp.h, sp.w), generator=g, device="cuda", dtype=torch.float32).half())
        ps.append(torch.rand((sp.c, sp.h, sp.w), generator=g, device="cuda", dtype=torch.float32).half())
    return Is, ps


def check_all(specs, Is, ps, *q_lists):
    """Every output of every image of each list of results (one per run)."""
    for k, (sp, dI, dp) in enumerate(zip(specs, Is, ps)):
        exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), sp.r, sp.s, sp.eps)
        tol = gpuutil.tolerance("f16", exp)
        for qs in q_lists:
            got = gpuutil.stored_f64(qs[k])
            assert np.all(np.abs(got - exp) <= tol), (k, sp, gpuutil.max_err(got, exp))
        if k % 64 == 63:
            print(f"  {k + 1} of {len(specs)} images checked", flush=True)


def test_full_256_image_batch():
    import torch
    specs = synth.batch_specs(256, seed=6)
    assert max(max(sp.h, sp.w) for sp in specs) > 1500  # the full-size draw, not a reduced one
    Is, ps = noise_images(torch, specs, seed=6)
    prs = [gfp.params(sp.r, sp.s, sp.eps) for sp in specs]
    out = {}
    for schedule in ("phases", "queue"):
        ctx = gfp.Context(0)
        ctx.set_batch_cfg(schedule, 24)
        out[schedule] = gfp.gf_fast_batched(Is, ps, prs, ctx=ctx)
        torch.cuda.synchronize()
        ctx.close()
        print(f"  {schedule}: batch done", flush=True)
    # the schedules differ in their box-mean tiles (48 rows under phases), so
    # each is held to the oracle
    check_all(specs, Is, ps, out["phases"], out["queue"])


def test_full_size_requests():
    import torch
    specs = [rq.spec for rq in synth.request_mix(12, qps=1000.0, seed=7)]
    specs.append(synth.ImageSpec(h=4000, w=6000, c=3, r=60, s=4, eps=1e-2, seed=0))  # 24 MP
    Is, ps = noise_images(torch, specs, seed=7)
    qs = [torch.empty_like(p) for p in ps]
    with gfp.Context(0, arena_bytes=4 << 30, max_inflight=64) as ctx:
        tickets = [ctx.gf_submit(dI, dp, q, sp.r, sp.s, sp.eps) for sp, dI, dp, q in zip(specs, Is, ps, qs)]
        for t in tickets:
            st, _ = ctx.gf_poll(t, wait_ms=-1)
            assert st == gfp.GF_OK
    torch.cuda.synchronize()
    print(f"  {len(specs)} requests served, {sum(sp.h * sp.w for sp in specs) / 1e6:.1f} MP", flush=True)
    check_all(specs, Is, ps, qs)
