"""ctypes wrapper around the FP64 CPU oracle (``gf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product path (the HIP
library and its binding) never imports this module.

Inputs are numpy arrays; they are converted to contiguous float64 (an exact
upcast for float32, float16 and bfloat16 values) before the call.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gf_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

NEAREST = 0
BILINEAR = 1
AREA = 2
_MODES = {"nearest": NEAREST, "bilinear": BILINEAR, "area": AREA, NEAREST: NEAREST, BILINEAR: BILINEAR,
          AREA: AREA}
# window means: clip-normalised, or over the image padded by edge replication / reflect-101
CLIP, REPLICATE, REFLECT101 = 0, 1, 2
_BORDERS = {"clip": CLIP, "replicate": REPLICATE, "reflect101": REFLECT101, CLIP: CLIP,
            REPLICATE: REPLICATE, REFLECT101: REFLECT101}

# IEEE double arithmetic as written: no fast-math, no FMA contraction.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off"]


def build(out: str = LIB, src: str = SRC) -> str:
    """Compile the oracle with gcc into a shared library (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


_DP = ctypes.POINTER(ctypes.c_double)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


class Oracle:
    """One loaded copy of the oracle library."""

    def __init__(self, libpath: str = LIB):
        lib = ctypes.CDLL(libpath)
        i, d = ctypes.c_int, ctypes.c_double
        sig = {
            "oracle_lowres_radius": [i, i],
            "oracle_lowres_size": [i, i],
            "oracle_box_mean": [_DP, i, i, i, _DP],
            "oracle_box_mean_border": [_DP, i, i, i, i, _DP],
            "oracle_subsample": [_DP, i, i, i, i, _DP],
            "oracle_upsample": [_DP, i, i, i, i, i, _DP],
            "oracle_coefficients": [_DP, _DP, i, i, i, d, _DP, _DP],
            "oracle_guided_filter": [_DP, _DP, i, i, i, i, d, _DP, _DP, _DP, _DP, _DP],
            "oracle_guided_filter_ex": [_DP, _DP, i, i, i, i, d, i, _DP, _DP, _DP, _DP, _DP],
            "oracle_fast_guided_filter": [_DP, _DP, i, i, i, i, i, d, i, _DP, _DP, _DP, _DP, _DP],
            "oracle_fast_guided_filter_ex": [_DP, _DP, i, i, i, i, i, d, i, i, _DP, _DP, _DP, _DP, _DP],
            "oracle_joint_upsample": [_DP, _DP, i, i, i, i, i, d, i, _DP],
            "oracle_joint_upsample_ex": [_DP, _DP, i, i, i, i, i, d, i, i, _DP],
            "oracle_detail_enhance": [_DP, _DP, ctypes.c_size_t, d, _DP],
            "oracle_fast_guided_filter_color": [_DP, _DP, i, i, i, i, i, d, i, i, _DP, _DP, _DP],
            "oracle_joint_upsample_color": [_DP, _DP, i, i, i, i, i, d, i, i, _DP],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        self.lib = lib
        self.path = libpath

    def lowres_radius(self, r: int, s: int) -> int:
        """r' = r/s rounded half up (at least 1 when r > 0)."""
        return int(self.lib.oracle_lowres_radius(int(r), int(s)))

    def lowres_size(self, n: int, s: int) -> int:
        return int(self.lib.oracle_lowres_size(int(n), int(s)))

    def box_mean(self, x, r: int, border="clip") -> np.ndarray:
        """(2r+1)^2 box mean of a 2-D array: clip-normalised, or over the
        image padded by replication / reflect-101."""
        x = _f64(x)
        h, w = x.shape
        out = np.empty_like(x)
        if _BORDERS[border] == CLIP:
            _check(self.lib.oracle_box_mean(_ptr(x), h, w, int(r), _ptr(out)), "oracle_box_mean")
        else:
            _check(self.lib.oracle_box_mean_border(_ptr(x), h, w, int(r), _BORDERS[border], _ptr(out)),
                   "oracle_box_mean_border")
        return out

    def subsample(self, x, s: int, mode="nearest") -> np.ndarray:
        x = _f64(x)
        h, w = x.shape
        out = np.empty((self.lowres_size(h, s), self.lowres_size(w, s)))
        _check(self.lib.oracle_subsample(_ptr(x), h, w, int(s), _MODES[mode], _ptr(out)),
               "oracle_subsample")
        return out

    def upsample(self, lo, s: int, h: int, w: int) -> np.ndarray:
        lo = _f64(lo)
        hl, wl = lo.shape
        out = np.empty((h, w))
        _check(self.lib.oracle_upsample(_ptr(lo), hl, wl, int(s), h, w, _ptr(out)),
               "oracle_upsample")
        return out

    def coefficients(self, I, p, r: int, eps: float):
        """a, b of Eqs. 2-3 for a single-channel p (Algorithm 1 steps 1-3)."""
        I, p = _f64(I), _f64(p)
        h, w = I.shape
        assert p.shape == (h, w)
        a, b = np.empty_like(I), np.empty_like(I)
        _check(self.lib.oracle_coefficients(_ptr(I), _ptr(p), h, w, int(r), float(eps),
                                            _ptr(a), _ptr(b)), "oracle_coefficients")
        return a, b

    @staticmethod
    def _as_chw(p, h, w):
        p = _f64(p)
        if p.ndim == 2:
            return np.ascontiguousarray(p.reshape(1, h, w)), True
        assert p.ndim == 3 and p.shape[1:] == (h, w), p.shape
        return p, False

    def guided_filter(self, I, p, r: int, eps: float, intermediates: bool = False, border="clip"):
        """Algorithm 1.  ``I`` is (h, w); ``p`` is (h, w) or (c, h, w).

        Returns q shaped like p, or (q, {a, b, mean_a, mean_b}).
        """
        I = _f64(I)
        h, w = I.shape
        p3, squeeze = self._as_chw(p, h, w)
        c = p3.shape[0]
        q = np.empty_like(p3)
        ex = ({k: np.empty_like(p3) for k in ("a", "b", "mean_a", "mean_b")}
              if intermediates else {})
        if _BORDERS[border] == CLIP:
            _check(self.lib.oracle_guided_filter(
                _ptr(I), _ptr(p3), c, h, w, int(r), float(eps), _ptr(q),
                _ptr(ex.get("a")), _ptr(ex.get("b")), _ptr(ex.get("mean_a")),
                _ptr(ex.get("mean_b"))), "oracle_guided_filter")
        else:
            _check(self.lib.oracle_guided_filter_ex(
                _ptr(I), _ptr(p3), c, h, w, int(r), float(eps), _BORDERS[border], _ptr(q),
                _ptr(ex.get("a")), _ptr(ex.get("b")), _ptr(ex.get("mean_a")),
                _ptr(ex.get("mean_b"))), "oracle_guided_filter_ex")
        if squeeze:
            q, ex = q[0], {k: v[0] for k, v in ex.items()}
        return (q, ex) if intermediates else q

    def fast_guided_filter(self, I, p, r: int, s: int, eps: float, mode="nearest",
                           intermediates: bool = False, border="clip"):
        """Algorithm 2.  Low-resolution intermediates (a, b, mean_a, mean_b)
        come back at ceil(h/s) x ceil(w/s) when ``intermediates`` is set."""
        I = _f64(I)
        h, w = I.shape
        p3, squeeze = self._as_chw(p, h, w)
        c = p3.shape[0]
        hl, wl = self.lowres_size(h, s), self.lowres_size(w, s)
        q = np.empty_like(p3)
        ex = ({k: np.empty((c, hl, wl)) for k in ("a", "b", "mean_a", "mean_b")}
              if intermediates else {})
        if _BORDERS[border] == CLIP and _MODES[mode] != AREA:
            _check(self.lib.oracle_fast_guided_filter(
                _ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps), _MODES[mode], _ptr(q),
                _ptr(ex.get("a")), _ptr(ex.get("b")), _ptr(ex.get("mean_a")),
                _ptr(ex.get("mean_b"))), "oracle_fast_guided_filter")
        else:
            _check(self.lib.oracle_fast_guided_filter_ex(
                _ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps), _MODES[mode], _BORDERS[border],
                _ptr(q), _ptr(ex.get("a")), _ptr(ex.get("b")), _ptr(ex.get("mean_a")),
                _ptr(ex.get("mean_b"))), "oracle_fast_guided_filter_ex")
        if squeeze:
            q, ex = q[0], {k: v[0] for k, v in ex.items()}
        return (q, ex) if intermediates else q


    def joint_upsample(self, I, p_lo, r: int, s: int, eps: float, mode="nearest", border="clip"):
        """Joint upsampling: ``p_lo`` (c, ceil(h/s), ceil(w/s)) or 2-D, guided
        by the full-resolution ``I`` (h, w).  Returns q at full resolution."""
        I = _f64(I)
        h, w = I.shape
        hl, wl = self.lowres_size(h, s), self.lowres_size(w, s)
        p_lo = _f64(p_lo)
        squeeze = p_lo.ndim == 2
        p3 = np.ascontiguousarray(p_lo.reshape(1, hl, wl)) if squeeze else p_lo
        assert p3.shape[1:] == (hl, wl), (p3.shape, hl, wl)
        c = p3.shape[0]
        q = np.empty((c, h, w))
        if _BORDERS[border] == CLIP and _MODES[mode] != AREA:
            _check(self.lib.oracle_joint_upsample(_ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps),
                                                  _MODES[mode], _ptr(q)), "oracle_joint_upsample")
        else:
            _check(self.lib.oracle_joint_upsample_ex(_ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps),
                                                     _MODES[mode], _BORDERS[border], _ptr(q)),
                   "oracle_joint_upsample_ex")
        return q[0] if squeeze else q

    def fast_guided_filter_color(self, I, p, r: int, s: int, eps: float, mode="nearest", border="clip",
                                 intermediates: bool = False):
        """Colour guidance: ``I`` is (3, h, w), ``p`` (h, w) or (c, h, w).
        s = 1 is the guided filter itself.  Low-res intermediates: a
        (c, 3, hl, wl) and b (c, hl, wl)."""
        I = np.ascontiguousarray(_f64(I))
        assert I.ndim == 3 and I.shape[0] == 3, I.shape
        h, w = I.shape[1:]
        p3, squeeze = self._as_chw(p, h, w)
        c = p3.shape[0]
        hl, wl = self.lowres_size(h, s), self.lowres_size(w, s)
        q = np.empty_like(p3)
        a = np.empty((c, 3, hl, wl)) if intermediates else None
        b = np.empty((c, hl, wl)) if intermediates else None
        _check(self.lib.oracle_fast_guided_filter_color(
            _ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps), _MODES[mode], _BORDERS[border], _ptr(q),
            _ptr(a), _ptr(b)), "oracle_fast_guided_filter_color")
        if squeeze:
            q = q[0]
            if intermediates:
                a, b = a[0], b[0]
        return (q, {"a": a, "b": b}) if intermediates else q

    def joint_upsample_color(self, I, p_lo, r: int, s: int, eps: float, mode="nearest", border="clip"):
        """Joint upsampling with a colour guide ``I`` (3, h, w); ``p_lo`` (c,
        ceil(h/s), ceil(w/s)) or 2-D.  Returns q at full resolution."""
        I = np.ascontiguousarray(_f64(I))
        assert I.ndim == 3 and I.shape[0] == 3, I.shape
        h, w = I.shape[1:]
        hl, wl = self.lowres_size(h, s), self.lowres_size(w, s)
        p_lo = _f64(p_lo)
        squeeze = p_lo.ndim == 2
        p3 = np.ascontiguousarray(p_lo.reshape(1, hl, wl)) if squeeze else p_lo
        assert p3.shape[1:] == (hl, wl), (p3.shape, hl, wl)
        c = p3.shape[0]
        q = np.empty((c, h, w))
        _check(self.lib.oracle_joint_upsample_color(_ptr(I), _ptr(p3), c, h, w, int(r), int(s), float(eps),
                                                    _MODES[mode], _BORDERS[border], _ptr(q)),
               "oracle_joint_upsample_color")
        return q[0] if squeeze else q

    def detail_enhance(self, p, q, gain: float):
        """e = q + gain (p - q), elementwise (p and q of one shape)."""
        p, q = _f64(p), _f64(q)
        assert p.shape == q.shape
        e = np.empty_like(q)
        _check(self.lib.oracle_detail_enhance(_ptr(p), _ptr(q), ctypes.c_size_t(q.size), float(gain), _ptr(e)),
               "oracle_detail_enhance")
        return e


_default: Oracle | None = None


def default() -> Oracle:
    """The oracle built from ``gf_oracle.c`` (compiled here if absent or stale)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _default = Oracle(LIB)
    return _default


def lowres_radius(r, s):
    return default().lowres_radius(r, s)


def lowres_size(n, s):
    return default().lowres_size(n, s)


def box_mean(x, r, border="clip"):
    return default().box_mean(x, r, border)


def subsample(x, s, mode="nearest"):
    return default().subsample(x, s, mode)


def upsample(lo, s, h, w):
    return default().upsample(lo, s, h, w)


def coefficients(I, p, r, eps):
    return default().coefficients(I, p, r, eps)


def guided_filter(I, p, r, eps, intermediates=False, border="clip"):
    return default().guided_filter(I, p, r, eps, intermediates, border)


def fast_guided_filter(I, p, r, s, eps, mode="nearest", intermediates=False, border="clip"):
    return default().fast_guided_filter(I, p, r, s, eps, mode, intermediates, border)


def joint_upsample(I, p_lo, r, s, eps, mode="nearest", border="clip"):
    return default().joint_upsample(I, p_lo, r, s, eps, mode, border)


def detail_enhance(p, q, gain):
    return default().detail_enhance(p, q, gain)


def fast_guided_filter_color(I, p, r, s, eps, mode="nearest", border="clip", intermediates=False):
    return default().fast_guided_filter_color(I, p, r, s, eps, mode, border, intermediates)


def joint_upsample_color(I, p_lo, r, s, eps, mode="nearest", border="clip"):
    return default().joint_upsample_color(I, p_lo, r, s, eps, mode, border)


def guided_filter_color(I, p, r, eps, border="clip"):
    return default().fast_guided_filter_color(I, p, r, 1, eps, "nearest", border)
