"""Helpers shared by the tests: library loading, tensor conversion, error
measures.  Holds none of the filter's arithmetic."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def ensure_built():
    """Build libgf.so when it is missing or older than any of its sources
    (csrc/, include/, the build script)."""
    import paper_1505_00996_amd as gfp
    from paper_1505_00996_amd import build
    if build.stale(gfp.LIB_PATH):
        build.build()
    return gfp


def torch_dtype(name: str):
    import torch
    return {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[name]


def to_device(x: np.ndarray, dtype: str = "f32"):
    """numpy float32 -> device tensor of the storage dtype (RNE cast on the host)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch_dtype(dtype))
    return t.to("cuda")


def stored_f64(t) -> np.ndarray:
    """Exact float64 copy of the stored values of a (host or device) tensor."""
    import torch
    return t.detach().to("cpu").to(torch.float64).numpy()


def batch_tiles(schedule: str, th: int) -> dict:
    """Tile shapes a batch with tile height th runs (radii small enough for
    48-row box tiles): box means take 48 rows under the phase schedule."""
    return dict(coeff_th=th, box_th=48 if schedule == "phases" else th)


def max_err(got: np.ndarray, exp: np.ndarray):
    d = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(exp, dtype=np.float64))
    i = int(np.argmax(d))
    return float(d.flat[i]), np.unravel_index(i, d.shape)


def bf16_half_ulp(x: np.ndarray) -> np.ndarray:
    """Half a bfloat16 unit in the last place at |x| (8 significant bits)."""
    return half_ulp("bf16", x)


_SIG_BITS = {"f32": 24, "f16": 11, "bf16": 8}
_MIN_EXP = {"f32": -126, "f16": -14, "bf16": -126}


def half_ulp(dtype: str, x) -> np.ndarray:
    """Half a unit in the last place of the storage format at |x| (the
    subnormal spacing below the normal range)."""
    ax = np.maximum(np.abs(np.asarray(x, dtype=np.float64)), np.finfo(np.float64).tiny)
    e = np.maximum(np.floor(np.log2(ax)), _MIN_EXP[dtype])
    return np.exp2(e - _SIG_BITS[dtype])


# FP32 error allowed before the store: the benchmark spec's bound of the FP32 path.
F32_TOL = 1e-5


def stated_tolerance(dtype: str, q_oracle):
    """The stated per-element bound: 1e-5 for FP32 storage, 2e-3 for 16-bit
    storage; for bfloat16 outputs with |q| >= 1 the rounding of the store
    alone can exceed 2e-3, so there the bound is half a bf16 ulp plus 1e-4."""
    if dtype == "f32":
        return F32_TOL
    if dtype == "f16":
        return np.full(np.shape(q_oracle), 2e-3)
    return np.where(np.abs(q_oracle) < 1.0, 2e-3, bf16_half_ulp(q_oracle) + 1e-4)


def ulp_gate(dtype: str, q_oracle):
    """What the arithmetic allows a 16-bit output: q is formed in FP32 within
    F32_TOL of the oracle and rounded once to nearest, so the stored value is
    within half an ulp of the FP32 q.  The half ulp is taken at
    |q_oracle| + F32_TOL, which covers an FP32 q that crossed into the next
    binade.  An FP32 compute error of order 1e-4 or more fails it, which the
    stated 2e-3 would not show."""
    if dtype == "f32":
        return F32_TOL
    return half_ulp(dtype, np.abs(q_oracle) + F32_TOL) + F32_TOL


def tolerance(dtype: str, q_oracle):
    """Per-element bound used by the parity tests: both the stated bound and
    the ulp gate hold (the gate is never the looser of the two)."""
    if dtype == "f32":
        return F32_TOL
    return np.minimum(stated_tolerance(dtype, q_oracle), ulp_gate(dtype, q_oracle))


def detail_tolerance(dtype: str, e_oracle, p, q_oracle, gain: float):
    """Bound for detail enhancement e = q + gain (p - q).  The kernel keeps q
    in FP32 (within F32_TOL of the oracle), forms p - q and one fused
    multiply-add in FP32 (two roundings, each at most 2^-24 relative) and
    rounds e once for storage.  So |e - e_oracle| <= |1 - gain| F32_TOL
    + 2^-24 (|gain| |p - q| + |e|) + half an ulp of the storage format at e.
    Rounding q to storage before forming e would add about |1 - gain| times
    half an ulp of q, which this bound rejects."""
    e_oracle = np.asarray(e_oracle, dtype=np.float64)
    f32 = 2.0 ** -24 * (abs(gain) * np.abs(np.asarray(p, dtype=np.float64) - q_oracle) + np.abs(e_oracle))
    slack = abs(1.0 - gain) * F32_TOL + f32 + 1e-7
    if dtype == "f32":
        return slack
    return half_ulp(dtype, np.abs(e_oracle) + slack) + slack


def round_to(dtype: str, x) -> np.ndarray:
    """Round FP64 values to the storage format (nearest even) and back."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    return t.to(torch_dtype(dtype)).to(torch.float64).numpy()


def ulp_distance(dtype: str, got, q_oracle) -> float:
    """Largest distance, in ulps of the storage format, between stored
    outputs and the oracle's value rounded to that format."""
    ref = round_to(dtype, q_oracle)
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref) / (2.0 * half_ulp(dtype, ref)))) \
        if np.size(ref) else 0.0


def split_16bit(q16, q32, exp):
    """The two errors of a 16-bit output, kept apart.  q32 is the same call
    run with FP32 storage on the stored inputs widened exactly to FP32: the
    16-bit kernels compute in FP32 from the same widened values, so the
    16-bit q must equal q32 rounded once to nearest even, bit for bit.  Then
    |q32 - oracle| is the compute error (within F32_TOL) and
    |q16 - oracle| the stored error.  Returns (compute error, stored error)."""
    import torch
    rounded = q32.to(q16.dtype)
    if not torch.equal(q16, rounded):
        n = int((q16 != rounded).sum())
        raise AssertionError(f"{n} 16-bit outputs differ from the FP32 path's q rounded once")
    pre = max_err(stored_f64(q32), exp)[0]
    assert pre <= F32_TOL, f"FP32 q before the store off by {pre:.3e}"
    return pre, max_err(stored_f64(q16), exp)[0]
