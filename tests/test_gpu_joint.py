"""Joint upsampling (gf_joint_upsample): a low-resolution input guided by the
full-resolution image, against the oracle, and bit for bit against gf_fast
when the low-resolution input is the nearest subsample of a full-res one
(GPU, through the C ABI)."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


def lowres_input(h, w, c, s, seed):
    """A smooth low-res field plus noise (not a subsample of anything)."""
    g = np.random.Generator(np.random.PCG64(seed))
    hl, wl = -(-h // s), -(-w // s)
    yy, xx = np.meshgrid(np.linspace(0, 1, hl), np.linspace(0, 1, wl), indexing="ij")
    out = np.stack([0.5 + 0.3 * np.sin(3 * yy + 2 * k) * np.cos(4 * xx - k) + g.normal(0, 0.05, (hl, wl))
                    for k in range(c)])
    return np.clip(out, 0, 1).astype(np.float32)


# (h, w, c, r, s, sub, dtype)
CASES = [(300, 400, 3, 16, 4, "nearest", "f32"), (257, 129, 1, 6, 2, "bilinear", "f32"),
         (511, 333, 3, 24, 8, "nearest", "f32"), (150, 151, 2, 9, 3, "bilinear", "f32"),
         (33, 47, 1, 0, 4, "nearest", "f32"), (1, 500, 1, 4, 4, "nearest", "f32"),
         (600, 800, 3, 16, 4, "bilinear", "f16"), (420, 380, 3, 12, 4, "nearest", "bf16")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_joint_matches_oracle(case):
    import torch
    h, w, c, r, s, sub, dt = case
    I = synth.photo_guide(h, w, seed=500 + h)
    p_lo = lowres_input(h, w, c, s, seed=600 + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p_lo, dt)
    q = gfp.gf_joint_upsample(dI, dp, r, s, 1e-3, sub)
    torch.cuda.synchronize()
    assert q.shape == (c, h, w)
    exp = oracle.joint_upsample(gpuutil.stored_f64(dI), gpuutil.stored_f64(dp), r, s, 1e-3, sub)
    got = gpuutil.stored_f64(q)
    assert np.all(np.abs(got - exp) <= gpuutil.tolerance(dt, exp)), (case, gpuutil.max_err(got, exp))


@pytest.mark.parametrize("dt", ["f32", "f16"])
def test_joint_of_nearest_subsample_equals_fast(dt):
    import torch
    h, w, c, r, s = 403, 517, 3, 12, 4
    I = synth.photo_guide(h, w, seed=7)
    p = synth.colour_input(I, c, seed=8)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    ys = torch.clamp(torch.arange(-(-h // s), device="cuda") * s + s // 2, max=h - 1)
    xs = torch.clamp(torch.arange(-(-w // s), device="cuda") * s + s // 2, max=w - 1)
    p_lo = dp[:, ys][:, :, xs].contiguous()
    ctx = gfp.Context(0)
    q_joint = gfp.gf_joint_upsample(dI, p_lo, r, s, 1e-3, ctx=ctx)
    q_fast = gfp.gf_fast(dI, dp, r, s, 1e-3, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(q_joint, q_fast)
    ctx.close()


def test_joint_12mp():
    """4000x3000 guide, 1000x750 RGB input (r = 16, s = 4), fp32."""
    import torch
    h, w, c, r, s = 3000, 4000, 3, 16, 4
    I, _ = synth.workload_12mp(h, w, c)
    p_lo = lowres_input(h, w, c, s, seed=11)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p_lo)
    q = gfp.gf_joint_upsample(dI, dp, r, s, 1e-3)
    torch.cuda.synchronize()
    exp = oracle.joint_upsample(I.astype(np.float64), p_lo.astype(np.float64), r, s, 1e-3)
    err = float(np.max(np.abs(q.double().cpu().numpy() - exp)))
    assert err <= 1e-5, err
