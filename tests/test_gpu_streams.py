"""Calls on a stream other than torch's current one (GPU, through the C
ABI): the binding allocates the workspace and q on the current stream and
marks them as used on the call's stream, so torch's caching allocator does
not hand their blocks out while the kernels still run there.  The result
equals the same call on the current stream, bit for bit."""
import pytest

import gpuutil
import synth

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


@pytest.mark.parametrize("as_handle", [False, True])
def test_side_stream_equals_current_stream(as_handle):
    import torch
    I = gpuutil.to_device(synth.photo_guide(1500, 2000, seed=21))
    p = gpuutil.to_device(synth.colour_input(synth.photo_guide(1500, 2000, seed=21), 3, seed=22))
    ref = gfp.gf_fast(I, p, 16, 4, 1e-3)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    stream = side.cuda_stream if as_handle else side
    outs = [gfp.gf_fast(I, p, 16, 4, 1e-3, stream=stream) for _ in range(4)]
    # allocate and fill on the current stream while `side` may still run
    junk = [torch.full((1 << 22,), float(k), device="cuda") for k in range(16)]
    side.synchronize()
    torch.cuda.synchronize()
    del junk
    assert all(torch.equal(q, ref) for q in outs)


def test_side_stream_batched_and_plain():
    import torch
    I = gpuutil.to_device(synth.photo_guide(300, 500, seed=23))
    p = gpuutil.to_device(synth.colour_input(synth.photo_guide(300, 500, seed=23), 2, seed=24))
    pr = gfp.params(8, 2, 1e-2)
    ref_b = gfp.gf_fast_batched([I, I], [p, p], [pr, pr])
    ref_p = gfp.gf_plain(I, p, 6, 1e-2)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    qb = gfp.gf_fast_batched([I, I], [p, p], [pr, pr], stream=side)
    qp = gfp.gf_plain(I, p, 6, 1e-2, stream=side)
    junk = [torch.full((1 << 20,), float(k), device="cuda") for k in range(16)]
    side.synchronize()
    del junk
    assert torch.equal(qb[0], ref_b[0]) and torch.equal(qb[1], ref_b[1]) and torch.equal(qp, ref_p)


def test_consecutive_images_on_two_streams():
    """Independent images alternated over two streams, each with its own
    context and workspace (the two-stream throughput that bench.py reports):
    the kernels of one image run beside the other's, and every output equals
    the same image filtered alone on the current stream."""
    import torch
    imgs = []
    for k in range(6):
        I = synth.photo_guide(600 + 40 * k, 800 - 24 * k, seed=31 + k)
        imgs.append((gpuutil.to_device(I), gpuutil.to_device(synth.colour_input(I, 1 + 2 * (k % 2), seed=41 + k))))
    refs = [gfp.gf_fast(I, p, 12, 4, 1e-3) for I, p in imgs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [gfp.Context(0), gfp.Context(0)]
    ws = [torch.empty(max(gfp.workspace_bytes(I.shape[-2], I.shape[-1], p.shape[0], 12, 4, 1e-3) for I, p in imgs),
                      dtype=torch.uint8, device="cuda") for _ in range(2)]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    outs = []
    for rep in range(3):
        for k, (I, p) in enumerate(imgs):
            outs.append((k, gfp.gf_fast(I, p, 12, 4, 1e-3, ctx=ctxs[k % 2], workspace=ws[k % 2],
                                        stream=streams[k % 2])))
    for st in streams:
        st.synchronize()
    for c in ctxs:
        c.close()
    bad = [k for k, q in outs if not torch.equal(q, refs[k])]
    assert not bad, f"images {bad} differ from the one-stream results"
