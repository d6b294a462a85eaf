"""Request interface (gf_submit / gf_poll): continuous batching with
admission by HBM footprint.  Each result equals the same request run alone,
whatever else was in flight with it (GPU, through the C ABI)."""
import time

import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def requests(n, seed=7, mp_hi=1.5):
    reqs = synth.request_mix(n, qps=1000.0, seed=seed, mp_lo=0.05, mp_hi=mp_hi)
    out = []
    for rq in reqs:
        I, p = synth.image_for(rq.spec)
        out.append((rq.spec, gpuutil.to_device(I, "f16"), gpuutil.to_device(p, "f16")))
    return out


def solo(ctx, spec, dI, dp):
    """The request alone: a batch of one under the same (default) batch
    configuration -- the tile height depends on the request's own radius only."""
    return gfp.gf_fast_batched([dI], [dp], [gfp.params(spec.r, spec.s, spec.eps)], ctx=ctx)[0]


def test_mix_equals_alone_and_oracle():
    import torch
    reqs = requests(20)
    ctx = gfp.Context(0, arena_bytes=1 << 30, max_inflight=64)
    qs, tickets = [], []
    for spec, dI, dp in reqs:
        q = torch.empty_like(dp)
        qs.append(q)
        tickets.append(ctx.gf_submit(dI, dp, q, spec.r, spec.s, spec.eps))
    stats = []
    for t in tickets:
        st, s = ctx.gf_poll(t, wait_ms=-1)
        assert st == gfp.GF_OK
        assert s.t_submit <= s.t_admit <= s.t_start <= s.t_done
        stats.append(s)
    ref = gfp.Context(0)
    for k, ((spec, dI, dp), q) in enumerate(zip(reqs, qs)):
        alone = solo(ref, spec, dI, dp)
        torch.cuda.synchronize()
        assert torch.equal(alone, q), (k, spec)
        if k % 4 == 0:
            exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), spec.r, spec.s,
                                            spec.eps)
            got = gpuutil.stored_f64(q)
            assert np.all(np.abs(got - exp) <= gpuutil.tolerance("f16", exp)), (k, spec)
    ref.close()
    ctx.close()


def test_small_arena_admits_as_memory_frees():
    """An arena that holds only about one request at a time still completes
    every request (they are admitted one after the other)."""
    import torch
    reqs = requests(8, seed=11, mp_hi=0.6)
    need = max(gfp.batched_workspace_bytes([dI], [dp], [gfp.params(sp.r, sp.s, sp.eps)])
               for sp, dI, dp in reqs)
    ctx = gfp.Context(0, arena_bytes=need + 4096, max_inflight=16)
    ref = gfp.Context(0)
    qs, tickets = [], []
    for spec, dI, dp in reqs:
        q = torch.empty_like(dp)
        qs.append(q)
        tickets.append(ctx.gf_submit(dI, dp, q, spec.r, spec.s, spec.eps))
    for t in tickets:
        assert ctx.gf_poll(t, wait_ms=-1)[0] == gfp.GF_OK
    for (spec, dI, dp), q in zip(reqs, qs):
        alone = solo(ref, spec, dI, dp)
        torch.cuda.synchronize()
        assert torch.equal(alone, q)
    ref.close()
    ctx.close()


def test_status_codes():
    import torch
    (spec, dI, dp), = requests(1, seed=3, mp_hi=0.3)
    q = torch.empty_like(dp)
    # too big for the arena: never admissible
    tiny = gfp.Context(0, arena_bytes=4096, max_inflight=4)
    with pytest.raises(gfp.GfError) as e:
        tiny.gf_submit(dI, dp, q, spec.r, spec.s, spec.eps)
    assert e.value.status == gfp.GF_ENOMEM
    tiny.close()
    ctx = gfp.Context(0, arena_bytes=1 << 28, max_inflight=2)
    t1 = ctx.gf_submit(dI, dp, q, spec.r, spec.s, spec.eps)
    q2 = torch.empty_like(dp)
    t2 = ctx.gf_submit(dI, dp, q2, spec.r, spec.s, spec.eps)
    q3 = torch.empty_like(dp)
    with pytest.raises(gfp.GfError) as e:
        ctx.gf_submit(dI, dp, q3, spec.r, spec.s, spec.eps)
    assert e.value.status == gfp.GF_EBUSY
    st, _ = ctx.gf_poll(t1, wait_ms=0)
    assert st in (gfp.GF_PENDING, gfp.GF_OK)
    if st == gfp.GF_PENDING:
        assert ctx.gf_poll(t1, wait_ms=-1)[0] == gfp.GF_OK
    with pytest.raises(gfp.GfError) as e:
        ctx.gf_poll(t1, wait_ms=0)  # retired
    assert e.value.status == gfp.GF_EINVAL
    assert ctx.gf_poll(t2, wait_ms=-1)[0] == gfp.GF_OK
    with pytest.raises(gfp.GfError) as e:
        ctx.gf_poll(987654321, wait_ms=0)
    assert e.value.status == gfp.GF_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(q, q2)
    ctx.close()


def test_radii_needing_different_tile_heights():
    """Requests whose r' = 2, 30, 33 get 24-, 16- and 8-row tiles on their
    own; interleaved, each still equals its own batch of one."""
    import torch
    specs = [(180, 260, 3, 8), (200, 240, 1, 120), (150, 300, 3, 8), (210, 220, 3, 132),
             (170, 250, 1, 8), (190, 230, 3, 120)]
    ctx = gfp.Context(0, arena_bytes=1 << 28, max_inflight=16)
    ref = gfp.Context(0)
    items = []
    for k, (h, w, c, r) in enumerate(specs):
        I = synth.photo_guide(h, w, seed=300 + k)
        p = synth.colour_input(I, c, seed=400 + k)
        dI, dp = gpuutil.to_device(I, "f16"), gpuutil.to_device(p, "f16")
        q = torch.empty_like(dp)
        items.append((h, w, c, r, dI, dp, q, ctx.gf_submit(dI, dp, q, r, 4, 1e-3)))
    for h, w, c, r, dI, dp, q, t in items:
        st, _ = ctx.gf_poll(t, wait_ms=-1)
        assert st == gfp.GF_OK
        alone = gfp.gf_fast_batched([dI], [dp], [gfp.params(r, 4, 1e-3)], ctx=ref)[0]
        torch.cuda.synchronize()
        assert torch.equal(alone, q), (h, w, c, r)
        exp = oracle.fast_guided_filter(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, 4, 1e-3)
        got = gpuutil.stored_f64(q)
        assert np.all(np.abs(got - exp) <= gpuutil.tolerance("f16", exp)), (h, w, c, r)
    ref.close()
    ctx.close()
