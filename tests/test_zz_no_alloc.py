"""gf_fast_noalloc (the entry point for callers that cannot allocate) on the
GPU through the C ABI: its q equals gf_fast's bit for bit (same kernels, same
tiles, only the workspace differs) and is within the stated tolerance of the
FP64 oracle; two calls in a row, the second smaller, so the second runs on the
fixed array still holding the first call's maps."""
import ctypes

import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def _pair(h, w, c, seed, dt, guide_c=1):
    if guide_c == 3:
        I = synth.colour_guide(h, w, seed=seed)
        p = synth.colour_input(I.mean(axis=0, dtype=np.float32), c, seed=seed + 1)
    else:
        I = synth.photo_guide(h, w, seed=seed)
        p = synth.colour_input(I, c, seed=seed + 1)
    return gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)


def _oracle(dI, dp, r, s, eps, sub, border):
    Is, ps = gpuutil.stored_f64(dI), gpuutil.stored_f64(dp)
    if dI.dim() == 3:
        return oracle.fast_guided_filter_color(Is, ps, r, s, eps, sub, border)
    return oracle.fast_guided_filter(Is, ps, r, s, eps, sub, border=border)


# Two calls in a row per case: (h, w, c, r, s, eps, sub, border, dtype, guide channels)
SEQUENCES = [
    [(1500, 2000, 3, 16, 4, 1e-3, "nearest", "clip", "f32", 1),
     (301, 257, 1, 8, 2, 1e-2, "bilinear", "clip", "f32", 1)],
    [(1200, 1600, 3, 32, 8, 1e-4, "nearest", "clip", "f16", 1),
     (333, 517, 3, 12, 4, 1e-3, "area", "reflect101", "f16", 1)],
    [(600, 800, 3, 16, 4, 1e-3, "nearest", "clip", "f32", 3),
     (150, 170, 1, 12, 3, 1e-3, "area", "replicate", "bf16", 3)],
]


@pytest.mark.parametrize("use_ctx", [False, True], ids=["no_ctx", "ctx"])
@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "_then_".join(f"{c[0]}x{c[1]}x{c[2]}" for c in s))
def test_noalloc_matches_gf_fast(seq, use_ctx):
    import torch
    ctx = gfp.Context(0) if use_ctx else None
    try:
        for k, (h, w, c, r, s, eps, sub, border, dt, gc) in enumerate(seq):
            print(f"noalloc call {k}: {h}x{w}x{c} guide {gc} r={r} s={s} eps={eps} {sub} {border} {dt} "
                  f"ctx={use_ctx}", flush=True)
            dI, dp = _pair(h, w, c, 700 + 31 * k + h, dt, gc)
            need = gfp.workspace_bytes(h, w, c, r, s, eps, sub, border, guide_c=gc)
            assert need <= gfp.NOALLOC_MAX_BYTES
            q = torch.empty_like(dp)
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            gfp.gf_fast_noalloc(dI, dp, r, s, eps, sub, q=q, ctx=ctx, border=border)
            assert torch.cuda.memory_allocated() == before  # the binding allocated nothing either
            ref = gfp.gf_fast(dI, dp, r, s, eps, sub, ctx=ctx, border=border)
            torch.cuda.synchronize()
            assert torch.equal(q, ref), f"call {k}: {int((q != ref).sum())} elements differ from gf_fast"
            exp = _oracle(dI, dp, r, s, eps, sub, border)
            got = gpuutil.stored_f64(q)
            assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), gpuutil.max_err(got, exp)
    finally:
        if ctx is not None:
            ctx.close()


def test_noalloc_on_a_side_stream_and_repeated():
    """The same call three times on a non-default stream, q cleared between
    calls: every result equals gf_fast's on the default stream."""
    import torch
    dI, dp = _pair(777, 1025, 3, 91, "f32")
    ref = gfp.gf_fast(dI, dp, 16, 4, 1e-3)
    side = torch.cuda.Stream()
    q = torch.empty_like(dp)
    for k in range(3):
        print(f"noalloc side-stream call {k}", flush=True)
        q.fill_(float("nan"))
        torch.cuda.synchronize()
        gfp.gf_fast_noalloc(dI, dp, 16, 4, 1e-3, q=q, stream=side)
        side.synchronize()
        assert torch.equal(q, ref)


def test_noalloc_rejects_maps_above_the_array():
    """A call whose low-res maps exceed the fixed array returns GF_ENOMEM
    before launching anything: q keeps its contents."""
    import torch
    h, w, c, r, s = 4096, 4096, 3, 8, 1  # 12 FP32 maps of 16 MP
    assert gfp.workspace_bytes(h, w, c, r, s, 1e-3) > gfp.NOALLOC_MAX_BYTES
    dI = torch.zeros(h, w, device="cuda")
    dp = torch.zeros(c, h, w, device="cuda")
    q = torch.full_like(dp, 7.0)
    pr = gfp.params(r, s, 1e-3)
    st = gfp.lib().gf_fast_noalloc(None, ctypes.byref(gfp.image(dI)), ctypes.byref(gfp.image(dp)),
                                   ctypes.byref(gfp.image(q)), ctypes.byref(pr), None)
    assert st == gfp.GF_ENOMEM
    assert "scratch" in gfp.last_error()
    torch.cuda.synchronize()
    assert bool((q == 7.0).all())
