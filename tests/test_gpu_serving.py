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
    ctx.set_tiles(dI, dp, spec.r, spec.s, spec.eps, dict(coeff_th=16, box_th=16))
    return gfp.gf_fast(dI, dp, spec.r, spec.s, spec.eps, ctx=ctx)


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
