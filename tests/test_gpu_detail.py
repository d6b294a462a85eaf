"""Detail enhancement (gf_detail_enhance): e = q + gain (p - q) against the
oracle; gain 0 gives gf_fast's q, gain 1 gives p (GPU, through the C ABI).

Tolerance (gpuutil.detail_tolerance): the kernel keeps q in FP32, within
1e-5 of the oracle, and forms e = q + gain (p - q) from it before the one
rounding to storage, so |e - e_oracle| <= |1 - gain| 1e-5 + two FP32
roundings + half an ulp of the storage format at e.  An epilogue that
rounded q to 16 bits first would be off by about |1 - gain| half an ulp of
q, which this bound rejects (tests/test_tolerance_power.py shows it on the
CPU)."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle

pytestmark = pytest.mark.gpu
gfp = gpuutil.ensure_built()


# (h, w, c, r, s, eps, gain, dtype): the paper's setting (r=16, eps=0.1^2, s=4, x5)
# in every storage format first
CASES = [(300, 400, 3, 16, 4, 1e-2, 5.0, "f32"), (400, 600, 3, 16, 4, 1e-2, 5.0, "f16"),
         (400, 600, 3, 16, 4, 1e-2, 5.0, "bf16"), (257, 129, 1, 8, 2, 1e-3, 3.0, "f32"),
         (150, 151, 3, 6, 1, 1e-2, 5.0, "f32"), (511, 333, 2, 24, 8, 1e-2, -1.0, "f32"),
         (222, 350, 3, 16, 4, 1e-2, 2.0, "bf16"), (181, 263, 1, 12, 2, 1e-3, 5.0, "f16")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_detail_matches_oracle(case):
    import torch
    h, w, c, r, s, eps, gain, dt = case
    I = synth.photo_guide(h, w, seed=700 + h)
    p = synth.colour_input(I, c, seed=800 + w)
    dI, dp = gpuutil.to_device(I, dt), gpuutil.to_device(p, dt)
    e = gfp.gf_detail_enhance(dI, dp, r, s, eps, gain)
    torch.cuda.synchronize()
    I64, p64 = gpuutil.stored_f64(dI), gpuutil.stored_f64(dp)
    q = oracle.fast_guided_filter(I64, p64, r, s, eps) if s > 1 else oracle.guided_filter(I64, p64, r, eps)
    exp = oracle.detail_enhance(p64, q, gain)
    got = gpuutil.stored_f64(e)
    tol = gpuutil.detail_tolerance(dt, exp, p64, q, gain)
    assert np.all(np.abs(got - exp) <= tol), (case, gpuutil.max_err(got, exp))


def test_detail_gain_end_points():
    import torch
    h, w, c = 301, 405, 3
    I = synth.photo_guide(h, w, seed=3)
    p = synth.colour_input(I, c, seed=4)
    dI, dp = gpuutil.to_device(I), gpuutil.to_device(p)
    ctx = gfp.Context(0)
    q = gfp.gf_fast(dI, dp, 16, 4, 1e-2, ctx=ctx)
    e0 = gfp.gf_detail_enhance(dI, dp, 16, 4, 1e-2, 0.0, ctx=ctx)
    e1 = gfp.gf_detail_enhance(dI, dp, 16, 4, 1e-2, 1.0, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(e0, q)  # q + 0 (p - q) is q
    d = (e1.double() - dp.double()).abs()
    assert float((d - 2.0 ** -24 * dp.double().abs().clamp_min(1.0)).max()) <= 0.0  # one rounding from p
    ctx.close()


def test_detail_rejects_non_finite_gain():
    I = gpuutil.to_device(synth.photo_guide(16, 16, seed=1))
    with pytest.raises(gfp.GfError):
        gfp.gf_detail_enhance(I, I.clone(), 2, 2, 1e-2, float("inf"))
