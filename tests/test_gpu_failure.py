"""Failure paths, forced from the host so that every kernel still ends
normally (GPU, through the C ABI):
  * gf_poll with a positive wait on a request that is still queued returns
    GF_ETIMEDOUT, and the request completes afterwards;
  * the queue schedule's bounded wait, limited to 0 polls on a context
    (gf_ctx_set_wait_limit), gives up at the first unfinished dependency:
    the kernels end, the batch's error word is set, gf_poll reports
    GF_EDEVICE for the request of that batch, and once the default limit is
    restored the same work completes with the bits gf_fast gives it with the
    queue schedule's tiles."""
import pytest

import gpuutil

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def _noise(shape, seed, dtype):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.rand(shape, generator=g, device="cuda", dtype=torch.float32).to(dtype)


def test_poll_times_out_on_queued_request():
    """Twelve plain-filter requests (s = 1, 3000x4000 gray fp16, r = 16) in an
    arena that holds five at a time: the last one is still queued after a
    1 ms wait."""
    import torch
    I = _noise((3000, 4000), 1, torch.float16)
    p = _noise((3000, 4000), 2, torch.float16)
    qs = [torch.empty_like(p) for _ in range(12)]
    torch.cuda.synchronize()  # the inputs are complete before gf_submit
    with gfp.Context(0, arena_bytes=1 << 30, max_inflight=32) as ctx:
        tickets = [ctx.gf_submit(I, p, q, 16, 1, 1e-3) for q in qs]
        print("submitted 12 plain-filter requests", flush=True)
        st, stats = ctx.gf_poll(tickets[-1], wait_ms=1)
        assert st == gfp.GF_ETIMEDOUT and stats is None
        for t in tickets:
            st, _ = ctx.gf_poll(t, wait_ms=-1)
            assert st == gfp.GF_OK
    ref = gfp.gf_fast_batched([I], [p], [gfp.params(16, 1, 1e-3)])[0]
    torch.cuda.synchronize()
    assert all(torch.equal(q, ref) for q in qs)


def _big_batch():
    """One 1536x2048 RGB fp16 image at s = 2, r = 20: 512 coefficient tiles,
    so under the queue schedule box-mean tasks are taken while coefficient
    tiles still run."""
    import torch
    I = _noise((1536, 2048), 3, torch.float16)
    p = _noise((3, 1536, 2048), 4, torch.float16)
    torch.cuda.synchronize()
    return I, p, gfp.params(20, 2, 1e-3)


def test_batched_wait_limit_gives_up_then_recovers():
    import torch
    I, p, pr = _big_batch()
    ctx = gfp.Context(0)
    ctx.set_batch_cfg("queue", 24)
    ws = torch.empty(gfp.batched_workspace_bytes([I], [p], [pr]), dtype=torch.uint8, device="cuda")
    ctx.set_wait_limit(0)
    print("queue schedule, wait limit 0", flush=True)
    gfp.gf_fast_batched([I], [p], [pr], ctx=ctx, workspace=ws)
    torch.cuda.synchronize()
    assert gfp.batched_wait_abandoned(ws)
    ctx.set_wait_limit(None)
    print("queue schedule, default wait limit", flush=True)
    q = gfp.gf_fast_batched([I], [p], [pr], ctx=ctx, workspace=ws)[0]
    torch.cuda.synchronize()
    assert not gfp.batched_wait_abandoned(ws)
    # the queue schedule runs {24, 24} tiles: q is gf_fast's with those tiles
    ctx.set_tiles(I, p, pr.r, pr.s, pr.eps, dict(coeff_th=24, box_th=24))
    solo = gfp.gf_fast(I, p, pr.r, pr.s, pr.eps, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(q, solo)
    ctx.close()


def test_served_wait_limit_reports_edevice():
    import torch
    I, p, pr = _big_batch()
    q = torch.empty_like(p)
    with gfp.Context(0, arena_bytes=1 << 30, max_inflight=8) as ctx:
        ctx.set_batch_cfg("queue", 24)
        ctx.set_wait_limit(0)
        t = ctx.gf_submit(I, p, q, pr.r, pr.s, pr.eps)
        with pytest.raises(gfp.GfError) as ei:
            ctx.gf_poll(t, wait_ms=-1)
        assert ei.value.status == gfp.GF_EDEVICE
        print("served request with wait limit 0: GF_EDEVICE", flush=True)
        ctx.set_wait_limit(None)
        t = ctx.gf_submit(I, p, q, pr.r, pr.s, pr.eps)
        st, _ = ctx.gf_poll(t, wait_ms=-1)
        assert st == gfp.GF_OK
        ref = gfp.gf_fast_batched([I], [p], [pr], ctx=ctx)[0]
        torch.cuda.synchronize()
        assert torch.equal(q, ref)
