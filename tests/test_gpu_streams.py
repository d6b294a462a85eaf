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
