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
    """Build libgf.so only when no built library is present."""
    import paper_1505_00996_amd as gfp
    if not os.path.exists(gfp.LIB_PATH):
        from paper_1505_00996_amd import build
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
    ax = np.maximum(np.abs(x), np.finfo(np.float32).tiny)
    return np.exp2(np.floor(np.log2(ax)) - 8)


def tolerance(dtype: str, q_oracle: np.ndarray):
    """Per-element bound: 1e-5 for FP32 storage, 2e-3 for 16-bit storage;
    for bfloat16 outputs with |q| >= 1 the rounding of the store alone can
    exceed 2e-3, so there the bound is half a bf16 ulp plus 1e-4."""
    if dtype == "f32":
        return 1e-5
    if dtype == "f16":
        return 2e-3
    return np.where(np.abs(q_oracle) < 1.0, 2e-3, bf16_half_ulp(q_oracle) + 1e-4)
