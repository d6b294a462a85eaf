"""The 16-bit tolerances of the GPU parity tests can tell compute error from
storage rounding (CPU only).

Each case builds, from the FP64 oracle, what a kernel would store under two
models, and runs the same bound the GPU tests apply:
  * the arithmetic the kernels do: q in FP32 (here the oracle's q rounded to
    FP32), rounded once to the storage format; for detail enhancement
    e = fma(gain, p - q, q) in FP32 from that FP32 q, rounded once;
  * a plausible slip: the detail epilogue formed from q already rounded to
    16 bits, or an FP32 compute error of order 1e-4 before the store.
The first must pass and the second must fail (on some element).  The
stated 2e-3 bound alone lets both slips through, which is why the GPU tests
also apply the per-element ulp gate."""
import numpy as np
import pytest

import gpuutil
import synth
from oracle import oracle


def _stored_inputs(dtype, h=120, w=160, c=3, seed=0):
    I = synth.photo_guide(h, w, seed=seed)
    p = synth.colour_input(I, c, seed=seed + 1)
    return gpuutil.round_to(dtype, I), gpuutil.round_to(dtype, p)


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_detail_bound_rejects_rounded_base(dtype):
    """The paper's detail setting (r = 16, eps = 0.1^2, s = 4, gain 5)."""
    gain = 5.0
    I, p = _stored_inputs(dtype)
    q = oracle.fast_guided_filter(I, p, 16, 4, 1e-2)
    e = oracle.detail_enhance(p, q, gain)
    tol = gpuutil.detail_tolerance(dtype, e, p, q, gain)
    # the kernel's arithmetic: FP32 q, FP32 difference, one fused multiply-add
    q32 = _f32(q)
    d32 = _f32(p - q32)
    good = gpuutil.round_to(dtype, _f32(gain * d32 + q32))
    assert np.all(np.abs(good - e) <= tol)
    # the slip: q rounded to storage before the epilogue
    q16 = gpuutil.round_to(dtype, q)
    bad = gpuutil.round_to(dtype, _f32(gain * _f32(p - q16) + q16))
    assert np.any(np.abs(bad - e) > tol)
    # the loose bound this replaces, |1 - gain| {2e-3, 4e-3} + half an ulp,
    # let the slip through
    old = abs(1 - gain) * {"f16": 2e-3, "bf16": 4e-3}[dtype] + gpuutil.half_ulp(dtype, e) + 1e-7
    assert np.all(np.abs(bad - e) <= old)


@pytest.mark.parametrize("dtype,err,stated_misses", [("f16", 1e-4, True), ("f16", 1e-3, True),
                                                     ("bf16", 2e-4, False)])
def test_ulp_gate_rejects_compute_error(dtype, err, stated_misses):
    """16-bit outputs of photo-like content at s = 4: the rounded FP32 q
    passes; an FP32 q off by `err` before the store fails the ulp gate.  For
    fp16 it stays inside the stated 2e-3 (half an fp16 ulp on [0.5, 1) is
    2.4e-4); for bf16 the stated bound is itself close to half an ulp."""
    I, p = _stored_inputs(dtype, 200, 260, 3, seed=5)
    q = oracle.fast_guided_filter(I, p, 16, 4, 1e-3)
    good = gpuutil.round_to(dtype, _f32(q))
    assert np.all(np.abs(good - q) <= gpuutil.tolerance(dtype, q))
    assert gpuutil.ulp_distance(dtype, good, q) <= 1.0
    bad = gpuutil.round_to(dtype, _f32(q + err))
    assert np.any(np.abs(bad - q) > gpuutil.tolerance(dtype, q))
    if stated_misses:
        assert np.all(np.abs(bad - q) <= gpuutil.stated_tolerance(dtype, q))


def test_half_ulp_values():
    """Half-ulp spacings at hand-checked points of each format."""
    assert gpuutil.half_ulp("f16", 0.75) == 2.0 ** -12      # 11 significant bits on [0.5, 1)
    assert gpuutil.half_ulp("f16", 1.0) == 2.0 ** -11
    assert gpuutil.half_ulp("f16", 1e-6) == 2.0 ** -25      # subnormal spacing 2^-24
    assert gpuutil.half_ulp("bf16", 0.75) == 2.0 ** -9      # 8 significant bits
    assert gpuutil.half_ulp("bf16", 1.5) == 2.0 ** -8
    assert gpuutil.half_ulp("f32", 0.75) == 2.0 ** -25
