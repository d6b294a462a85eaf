"""Maximum sizes: one 40000 x 54000 image (2.16e9 pixels per plane, past
2^31 elements, so every row and plane offset needs 64-bit arithmetic)
through the per-image fast and plain filters and the batched kernels, fp16
(GPU, through the C ABI).

The outputs are checked on crops.  The filter is local: q at a pixel reads
low-res rows and columns within 2r'+1 of its upsampling taps, each of which
samples full-res pixels within s of it.  So the oracle run on a crop whose
origin lies on the low-res grid (a multiple of s) gives the image's own
result at every pixel at least (2r'+4)s from a crop edge that is not an
image edge.  One crop straddles the row where the element offset y*W
passes 2^31."""
import numpy as np
import pytest

import gpuutil
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()

H, W = 40000, 54000
ROW_2_31 = -(-(1 << 31) // W)  # first row whose offset y*W is at least 2^31


def crops():
    """(y0, y1, x0, x1): corners, an edge, and the 2^31 crossing; origins and
    interior ends on multiples of 4 (the largest s used here)."""
    n = 352
    yc = (ROW_2_31 - n // 2) // 4 * 4
    return [(0, n, 0, n), (H - n, H, W - n, W), (20000, 20000 + n, W - n, W), (yc, yc + n, 26000, 26000 + n)]


@pytest.fixture(scope="module")
def big():
    import torch
    assert H * W > (1 << 31) and crops()[3][0] + 48 < ROW_2_31 < crops()[3][1] - 48
    g = torch.Generator(device="cuda")
    g.manual_seed(2024)
    I = torch.empty((H, W), dtype=torch.float16, device="cuda")
    p = torch.empty((1, H, W), dtype=torch.float16, device="cuda")
    for y in range(0, H, 2000):  # seeded noise, made in bands to bound the FP32 temporaries
        I[y:y + 2000].copy_(torch.rand((2000, W), generator=g, device="cuda"))
        p[0, y:y + 2000].copy_(torch.rand((2000, W), generator=g, device="cuda"))
    torch.cuda.synchronize()
    print(f"  {H}x{W} fp16 guide and input made", flush=True)
    yield I, p
    del I, p
    torch.cuda.empty_cache()


def check_crops(I, p, q, r, s, eps):
    R = oracle.lowres_radius(r, s)
    m = (2 * R + 4) * s
    for y0, y1, x0, x1 in crops():
        cI, cp = gpuutil.stored_f64(I[y0:y1, x0:x1]), gpuutil.stored_f64(p[:, y0:y1, x0:x1])
        exp = oracle.fast_guided_filter(cI, cp, r, s, eps) if s > 1 else oracle.guided_filter(cI, cp, r, eps)
        got = gpuutil.stored_f64(q[:, y0:y1, x0:x1])
        iy = slice(0 if y0 == 0 else m, (y1 - y0) if y1 == H else (y1 - y0) - m)
        ix = slice(0 if x0 == 0 else m, (x1 - x0) if x1 == W else (x1 - x0) - m)
        g, e = got[:, iy, ix], exp[:, iy, ix]
        assert g.size >= 256 * 256
        assert np.all(np.abs(g - e) <= gpuutil.tolerance("f16", e)), ((y0, x0), s, gpuutil.max_err(g, e))


def test_max_size_fast_and_batched(big):
    import torch
    I, p = big
    q = gfp.gf_fast(I, p, 16, 4, 1e-3)
    torch.cuda.synchronize()
    print("  gf_fast done", flush=True)
    check_crops(I, p, q, 16, 4, 1e-3)
    qb = gfp.gf_fast_batched([I], [p], [gfp.params(16, 4, 1e-3)])[0]
    torch.cuda.synchronize()
    print("  gf_fast_batched done", flush=True)
    assert torch.equal(q, qb)  # same tiles (24 rows at r' = 4): the same bits
    del q, qb


def test_max_size_plain(big):
    import torch
    I, p = big
    q = gfp.gf_plain(I, p, 16, 1e-3)
    torch.cuda.synchronize()
    print("  gf_plain done", flush=True)
    check_crops(I, p, q, 16, 1, 1e-3)
    del q
