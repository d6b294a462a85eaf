"""Python binding of libgf.so, the MI355X guided-filter library (include/gf.h).

Argument marshalling only: torch tensors on the GPU are described to the C ABI
as ``gf_image`` views (pointer, dtype, shape, strides in elements) and the
current torch stream is passed as the ``hipStream_t``; every step of the
filter runs in the library's HIP kernels.  The functions carry the names of
the C entry points: ``gf_plain``, ``gf_fast``, ``gf_fast_batched``,
``gf_submit`` and ``gf_poll`` (the latter two through ``Context``).

There is no fallback: if libgf.so is missing or fails to load, every call
raises.  Build it with ``python -m paper_1505_00996_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgf.so")

GF_OK, GF_PENDING = 0, 1
GF_EINVAL, GF_ENOMEM, GF_EBUSY, GF_ENOTSUP, GF_EDEVICE, GF_ETIMEDOUT = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "GF_OK", 1: "GF_PENDING", -1: "GF_EINVAL", -2: "GF_ENOMEM", -3: "GF_EBUSY",
                -4: "GF_ENOTSUP", -5: "GF_EDEVICE", -6: "GF_ETIMEDOUT"}
GF_F32, GF_F16, GF_BF16 = 0, 1, 2
GF_BORDER_CLIP, GF_BORDER_REPLICATE, GF_BORDER_REFLECT101 = 0, 1, 2
BORDERS = {"clip": GF_BORDER_CLIP, "replicate": GF_BORDER_REPLICATE, "reflect101": GF_BORDER_REFLECT101}
GF_SUB_NEAREST, GF_SUB_BILINEAR, GF_SUB_AREA = 0, 1, 2
SUBSAMPLE = {"nearest": GF_SUB_NEAREST, "bilinear": GF_SUB_BILINEAR, "area": GF_SUB_AREA}

# Every symbol include/gf.h declares.
EXPORTS = ("gf_ctx_create", "gf_ctx_destroy", "gf_last_error", "gf_workspace_bytes", "gf_plain",
           "gf_fast", "gf_batched_workspace_bytes", "gf_fast_batched", "gf_submit", "gf_poll",
           "gf_ctx_profile", "gf_ctx_profile_read", "gf_ctx_set_tiles", "gf_tune",
           "gf_ctx_save_tuning", "gf_ctx_load_tuning", "gf_batch_create", "gf_batch_launch",
           "gf_batch_destroy", "gf_ctx_set_batch_cfg", "gf_tune_batched", "gf_footprint_bytes", "gf_joint_upsample",
           "gf_detail_enhance", "gf_workspace_bytes_guide", "gf_ctx_set_wait_limit", "gf_fast_noalloc", "gf_ctx_set_fusion")
KERNELS = ("coeff", "box", "output", "batched", "area")


class gf_image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int), ("c", ctypes.c_int32),
                ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("row_stride", ctypes.c_int64),
                ("plane_stride", ctypes.c_int64)]


class gf_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("s", ctypes.c_int32), ("eps", ctypes.c_double),
                ("border", ctypes.c_int), ("sub", ctypes.c_int)]


class gf_req_stats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class gf_kernel_time(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("launches", ctypes.c_int64)]


class gf_tiles(ctypes.Structure):
    _fields_ = [("coeff_th", ctypes.c_int32), ("box_th", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gf_tune_result(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tiles", gf_tiles), ("ms", ctypes.c_double)]


GF_FUSE_OFF, GF_FUSE_AUTO, GF_FUSE_ON = 0, 1, 2
FUSION = {"off": GF_FUSE_OFF, "auto": GF_FUSE_AUTO, "on": GF_FUSE_ON}

GF_BATCH_PHASES, GF_BATCH_QUEUE = 0, 1
SCHEDULES = {"phases": GF_BATCH_PHASES, "queue": GF_BATCH_QUEUE}


class gf_batch_cfg(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("tile_h", ctypes.c_int32)]

    def as_dict(self):
        return {"schedule": {v: k for k, v in SCHEDULES.items()}[self.schedule], "tile_h": self.tile_h}


class gf_batch_tune_result(ctypes.Structure):
    _fields_ = [("cfg", gf_batch_cfg), ("ms", ctypes.c_double)]


class GfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgf.so (raises if it has not been built).

    torch is imported first so that libgf.so binds to the HIP runtime torch
    already loaded (same soname): the streams and device pointers torch hands
    over are only valid in that runtime, and a second HIP runtime in the
    process would not know them."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime before libgf.so)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_1505_00996_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, VP, SZ = (ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_size_t)
        img_p, par_p = P(gf_image), P(gf_params)
        sig = {
            "gf_ctx_create": (ctypes.c_int, [P(VP), ctypes.c_int, SZ, ctypes.c_int]),
            "gf_ctx_destroy": (None, [VP]),
            "gf_last_error": (ctypes.c_char_p, [VP]),
            "gf_workspace_bytes": (SZ, [I32, I32, I32, par_p]),
            "gf_workspace_bytes_guide": (SZ, [I32, I32, I32, I32, par_p]),
            "gf_plain": (ctypes.c_int, [VP, img_p, img_p, img_p, I32, D, ctypes.c_int, VP, SZ, VP]),
            "gf_fast": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, VP, SZ, VP]),
            "gf_fast_noalloc": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, VP]),
            "gf_joint_upsample": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, VP, SZ, VP]),
            "gf_detail_enhance": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, D, VP, SZ, VP]),
            "gf_batched_workspace_bytes": (SZ, [I32, img_p, img_p, par_p]),
            "gf_fast_batched": (ctypes.c_int, [VP, I32, img_p, img_p, img_p, par_p, VP, SZ, VP]),
            "gf_submit": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, P(ctypes.c_uint64)]),
            "gf_poll": (ctypes.c_int, [VP, ctypes.c_uint64, I32, P(gf_req_stats)]),
            "gf_ctx_profile": (ctypes.c_int, [VP, ctypes.c_int]),
            "gf_ctx_profile_read": (ctypes.c_int, [VP, P(gf_kernel_time)]),
            "gf_ctx_set_tiles": (ctypes.c_int, [VP, ctypes.c_int, I32, I32, I32, par_p, P(gf_tiles)]),
            "gf_tune": (ctypes.c_int, [VP, img_p, img_p, img_p, par_p, VP, SZ, VP, I32, P(gf_tiles),
                                       P(gf_tune_result), I32, P(I32)]),
            "gf_ctx_save_tuning": (ctypes.c_int, [VP, ctypes.c_char_p]),
            "gf_ctx_load_tuning": (ctypes.c_int, [VP, ctypes.c_char_p]),
            "gf_batch_create": (ctypes.c_int, [VP, I32, img_p, img_p, img_p, par_p, VP, SZ, VP, P(VP)]),
            "gf_batch_launch": (ctypes.c_int, [VP, VP]),
            "gf_batch_destroy": (None, [VP]),
            "gf_ctx_set_batch_cfg": (ctypes.c_int, [VP, P(gf_batch_cfg)]),
            "gf_ctx_set_wait_limit": (ctypes.c_int, [VP, I64]),
            "gf_ctx_set_fusion": (ctypes.c_int, [VP, ctypes.c_int]),
            "gf_footprint_bytes": (SZ, [I32, I32, I32, ctypes.c_int, par_p]),
            "gf_tune_batched": (ctypes.c_int, [VP, I32, img_p, img_p, img_p, par_p, VP, SZ, VP, I32,
                                               P(gf_batch_cfg), P(gf_batch_tune_result), I32, P(I32)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error(ctx=None) -> str:
    return (lib().gf_last_error(ctx._h if ctx else None) or b"").decode()


def _check(st: int, ctx=None) -> int:
    if st < 0:
        raise GfError(st, last_error(ctx))
    return st


def _dtype_code(t) -> int:
    import torch
    codes = {torch.float32: GF_F32, torch.float16: GF_F16, torch.bfloat16: GF_BF16}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32, float16 or bfloat16")
    return codes[t.dtype]


def image(t) -> gf_image:
    """Describe a (H, W) or (C, H, W) device tensor as a gf_image (no copy)."""
    if not t.is_cuda:
        raise ValueError("gf images must be GPU tensors")
    if t.dim() == 2:
        c, (h, w) = 1, t.shape
        rs, ps = t.stride(0), t.stride(0) * h
        if t.stride(1) != 1:
            raise ValueError("rows must be contiguous (stride 1 along W)")
    elif t.dim() == 3:
        c, h, w = t.shape
        ps, rs, cs = t.stride()
        if cs != 1:
            raise ValueError("rows must be contiguous (stride 1 along W)")
    else:
        raise ValueError("expected a (H, W) or (C, H, W) tensor")
    return gf_image(t.data_ptr(), _dtype_code(t), c, h, w, rs, ps)


def params(r: int, s: int, eps: float, sub: str | int = "nearest", border: str | int = "clip") -> gf_params:
    """Filter parameters; ``sub`` in SUBSAMPLE, ``border`` in BORDERS (or their codes)."""
    return gf_params(int(r), int(s), float(eps), BORDERS[border] if isinstance(border, str) else int(border),
                     SUBSAMPLE[sub] if isinstance(sub, str) else int(sub))


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_bytes(h: int, w: int, c: int, r: int, s: int, eps: float, sub="nearest", border="clip",
                    guide_c: int = 1) -> int:
    return int(lib().gf_workspace_bytes_guide(h, w, guide_c, c, ctypes.byref(params(r, s, eps, sub, border))))


def _guide_c(I) -> int:
    return 1 if I.dim() == 2 else int(I.shape[0])


def _workspace(nbytes: int, device):
    import torch
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


def _used_on(stream, *tensors):
    """Tensors allocated here on torch's current stream but written by work
    enqueued on `stream`: tell torch's caching allocator, so that their
    blocks are not handed to another allocation before that work is done."""
    if stream is None:
        return
    import torch
    s = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream))
    if s.cuda_stream == torch.cuda.current_stream().cuda_stream:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def _out_like(p, q):
    import torch
    if q is None:
        return torch.empty_like(p, memory_format=torch.contiguous_format)
    return q


def gf_fast(I, p, r: int, s: int, eps: float, sub: str = "nearest", q=None, ctx=None,
            workspace=None, stream=None, border: str = "clip"):
    """Algorithm 2 on the GPU: returns q (shape of p).  ``I`` is (H, W), or
    (3, H, W) for a colour guide; ``p`` is (H, W) or (C, H, W); same dtype
    (float32 / float16 / bfloat16)."""
    own_q = q is None
    q = _out_like(p, q)
    pr = params(r, s, eps, sub, border)
    h, w = I.shape[-2:]
    c = 1 if p.dim() == 2 else p.shape[0]
    need = int(lib().gf_workspace_bytes_guide(h, w, _guide_c(I), c, ctypes.byref(pr)))
    own_ws = workspace is None
    if own_ws:
        workspace = _workspace(need, p.device)
    _used_on(stream, workspace if own_ws else None, q if own_q else None)
    _check(lib().gf_fast(ctx._h if ctx else None, ctypes.byref(image(I)), ctypes.byref(image(p)),
                         ctypes.byref(image(q)), ctypes.byref(pr), ctypes.c_void_p(workspace.data_ptr()),
                         workspace.numel() * workspace.element_size(), _stream(stream)), ctx)
    return q


# Size of the fixed device array gf_fast_noalloc keeps its low-res maps in.
NOALLOC_MAX_BYTES = 64 << 20


def gf_fast_noalloc(I, p, r: int, s: int, eps: float, sub: str = "nearest", q=None, ctx=None, stream=None,
                    border: str = "clip"):
    """gf_fast without a workspace: the library keeps the low-res maps in a
    fixed per-GPU device array (NOALLOC_MAX_BYTES).  With ``q`` given the call
    allocates nothing; calls that overlap on one GPU race on that array."""
    own_q = q is None
    q = _out_like(p, q)
    _used_on(stream, q if own_q else None)
    _check(lib().gf_fast_noalloc(ctx._h if ctx else None, ctypes.byref(image(I)), ctypes.byref(image(p)),
                                 ctypes.byref(image(q)), ctypes.byref(params(r, s, eps, sub, border)),
                                 _stream(stream)), ctx)
    return q


def gf_joint_upsample(I, p_low, r: int, s: int, eps: float, sub: str = "nearest", q=None, ctx=None,
                      workspace=None, stream=None, border: str = "clip"):
    """Joint upsampling: ``p_low`` (c, ceil(h/s), ceil(w/s)) or 2-D, guided by
    ``I`` (h, w); returns q at full resolution (c, h, w) or (h, w)."""
    h, w = I.shape[-2:]
    own_q = q is None
    if own_q:
        import torch
        q = torch.empty(p_low.shape[:-2] + (h, w), dtype=p_low.dtype, device=p_low.device)
    pr = params(r, s, eps, sub, border)
    c = 1 if p_low.dim() == 2 else p_low.shape[0]
    own_ws = workspace is None
    if own_ws:
        workspace = _workspace(int(lib().gf_workspace_bytes_guide(h, w, _guide_c(I), c, ctypes.byref(pr))), I.device)
    _used_on(stream, workspace if own_ws else None, q if own_q else None)
    _check(lib().gf_joint_upsample(ctx._h if ctx else None, ctypes.byref(image(I)), ctypes.byref(image(p_low)),
                                   ctypes.byref(image(q)), ctypes.byref(pr), ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel() * workspace.element_size(), _stream(stream)), ctx)
    return q


def gf_detail_enhance(I, p, r: int, s: int, eps: float, gain: float, sub: str = "nearest", e=None, ctx=None,
                      workspace=None, stream=None, border: str = "clip"):
    """Detail enhancement: e = q + gain (p - q) with q the fast filter of p
    (plain at s = 1).  Returns e (shape of p)."""
    own_e = e is None
    e = _out_like(p, e)
    pr = params(r, s, eps, sub, border)
    h, w = I.shape[-2:]
    c = 1 if p.dim() == 2 else p.shape[0]
    own_ws = workspace is None
    if own_ws:
        workspace = _workspace(int(lib().gf_workspace_bytes_guide(h, w, _guide_c(I), c, ctypes.byref(pr))), p.device)
    _used_on(stream, workspace if own_ws else None, e if own_e else None)
    _check(lib().gf_detail_enhance(ctx._h if ctx else None, ctypes.byref(image(I)), ctypes.byref(image(p)),
                                   ctypes.byref(image(e)), ctypes.byref(pr), float(gain),
                                   ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                   _stream(stream)), ctx)
    return e


def gf_plain(I, p, r: int, eps: float, q=None, ctx=None, workspace=None, stream=None, border: str = "clip"):
    """Algorithm 1 on the GPU (full resolution): returns q (shape of p).
    ``I`` is (H, W), or (3, H, W) for a colour guide."""
    own_q = q is None
    q = _out_like(p, q)
    pr = params(r, 1, eps, "nearest", border)
    h, w = I.shape[-2:]
    c = 1 if p.dim() == 2 else p.shape[0]
    need = int(lib().gf_workspace_bytes_guide(h, w, _guide_c(I), c, ctypes.byref(pr)))
    own_ws = workspace is None
    if own_ws:
        workspace = _workspace(need, p.device)
    _used_on(stream, workspace if own_ws else None, q if own_q else None)
    _check(lib().gf_plain(ctx._h if ctx else None, ctypes.byref(image(I)), ctypes.byref(image(p)),
                          ctypes.byref(image(q)), int(r), float(eps), pr.border,
                          ctypes.c_void_p(workspace.data_ptr()),
                          workspace.numel() * workspace.element_size(), _stream(stream)), ctx)
    return q


def _arrays(Is, ps, qs, prs):
    n = len(Is)
    if not (len(ps) == len(qs) == len(prs) == n):
        raise ValueError("I, p, q and params lists must have the same length")
    return ((gf_image * n)(*[image(t) for t in Is]), (gf_image * n)(*[image(t) for t in ps]),
            (gf_image * n)(*[image(t) for t in qs]), (gf_params * n)(*prs))


def footprint_bytes(h: int, w: int, c: int, r: int, s: int, eps: float, dtype: int = GF_F32,
                    sub="nearest", border="clip") -> int:
    """Arena bytes one request of this shape occupies (gf_footprint_bytes)."""
    return int(lib().gf_footprint_bytes(h, w, c, dtype, ctypes.byref(params(r, s, eps, sub, border))))


def batched_workspace_bytes(Is, ps, prs) -> int:
    n = len(Is)
    aI, ap, _, apr = _arrays(Is, ps, ps, prs)
    return int(lib().gf_batched_workspace_bytes(n, aI, ap, apr))


def gf_fast_batched(Is, ps, prs, qs=None, ctx=None, workspace=None, stream=None):
    """Algorithm 2 for a list of images in one persistent launch.  ``prs`` is
    a list of ``params(r, s, eps, sub)``.  Returns the list of outputs."""
    own_q = qs is None
    if own_q:
        qs = [_out_like(p, None) for p in ps]
    n = len(Is)
    aI, ap, aq, apr = _arrays(Is, ps, qs, prs)
    own_ws = workspace is None
    if own_ws:
        workspace = _workspace(lib().gf_batched_workspace_bytes(n, aI, ap, apr), ps[0].device)
    _used_on(stream, workspace if own_ws else None, *(qs if own_q else ()))
    _check(lib().gf_fast_batched(ctx._h if ctx else None, n, aI, ap, aq, apr,
                                 ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size(), _stream(stream)), ctx)
    return qs


def batched_wait_abandoned(workspace) -> bool:
    """After a batched launch has completed: True if some tile gave up
    waiting for the previous phase of its image (its outputs are then
    incomplete).  Reads word 1 of the batch workspace."""
    import torch
    return bool(workspace[4:8].cpu().view(torch.int32).item())


class Batch:
    """gf_batch: a planned batch whose launch() only enqueues kernels, so it
    can be captured into a HIP graph (torch.cuda.graph) and replayed.  Keeps
    I, p, q and the workspace alive; each launch reads the current I, p."""

    def __init__(self, Is, ps, prs, qs=None, ctx=None, workspace=None, stream=None):
        if qs is None:
            qs = [_out_like(p, None) for p in ps]
        n = len(Is)
        aI, ap, aq, apr = _arrays(Is, ps, qs, prs)
        if workspace is None:
            workspace = _workspace(lib().gf_batched_workspace_bytes(n, aI, ap, apr), ps[0].device)
        h = ctypes.c_void_p()
        _check(lib().gf_batch_create(ctx._h if ctx else None, n, aI, ap, aq, apr,
                                     ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel() * workspace.element_size(), _stream(stream),
                                     ctypes.byref(h)), ctx)
        self._h = h
        self.Is, self.ps, self.qs, self.workspace = list(Is), list(ps), qs, workspace

    def launch(self, stream=None):
        _check(lib().gf_batch_launch(self._h, _stream(stream)))
        return self.qs

    def close(self):
        if getattr(self, "_h", None):
            lib().gf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class ReqStats:
    t_submit: float
    t_admit: float
    t_start: float
    t_done: float


class Context:
    """A gf_ctx: device, optional request arena (gf_submit / gf_poll)."""

    def __init__(self, device: int = 0, arena_bytes: int = 0, max_inflight: int = 0):
        h = ctypes.c_void_p()
        _check(lib().gf_ctx_create(ctypes.byref(h), int(device), int(arena_bytes), int(max_inflight)))
        self._h = h
        self._keep = {}

    def close(self):
        if self._h:
            lib().gf_ctx_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Record HIP events around every kernel this context launches."""
        _check(lib().gf_ctx_profile(self._h, int(bool(enable))), self)

    def profile_read(self) -> dict:
        """{kernel: (total_ms, launches)} since the last read (waits for the events)."""
        out = (gf_kernel_time * len(KERNELS))()
        _check(lib().gf_ctx_profile_read(self._h, out), self)
        return {k: (out[i].total_ms, out[i].launches) for i, k in enumerate(KERNELS)}

    def set_tiles(self, I, p, r: int, s: int, eps: float, tiles: dict | None, sub: str = "nearest"):
        """Pin tile shapes for the class of this problem (None: unpin)."""
        h, w = I.shape[-2:]
        c = 1 if p.dim() == 2 else p.shape[0]
        t = gf_tiles(**tiles) if tiles is not None else None
        _check(lib().gf_ctx_set_tiles(self._h, _dtype_code(I), h, w, c,
                                      ctypes.byref(params(r, s, eps, sub)),
                                      ctypes.byref(t) if t is not None else None), self)

    def tune(self, I, p, r: int, s: int, eps: float, sub: str = "nearest", q=None, reps: int = 5,
             stream=None, border: str = "clip"):
        """Autotune the window-sum kernels for this problem's class.
        Returns (best tiles dict, [(kernel, tiles dict, ms), ...])."""
        q = _out_like(p, q)
        h, w = I.shape[-2:]
        c = 1 if p.dim() == 2 else p.shape[0]
        pr = params(r, s, eps, sub, border)
        ws = _workspace(lib().gf_workspace_bytes(h, w, c, ctypes.byref(pr)), p.device)
        best = gf_tiles()
        res = (gf_tune_result * 64)()
        n = ctypes.c_int32()
        _check(lib().gf_tune(self._h, ctypes.byref(image(I)), ctypes.byref(image(p)),
                             ctypes.byref(image(q)), ctypes.byref(pr), ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream(stream), int(reps), ctypes.byref(best), res, 64,
                             ctypes.byref(n)), self)
        rows = [(KERNELS[res[i].kernel], res[i].tiles.as_dict(), res[i].ms) for i in range(n.value)]
        return best.as_dict(), rows

    def save_tuning(self, path: str):
        _check(lib().gf_ctx_save_tuning(self._h, path.encode()), self)

    def load_tuning(self, path: str):
        _check(lib().gf_ctx_load_tuning(self._h, path.encode()), self)

    def set_fusion(self, mode: str = "auto"):
        """Box means fused into the output pass: "auto" (the default: small
        problems), "on" (wherever it applies) or "off" (the separate
        box-mean pass); the same bits either way."""
        _check(lib().gf_ctx_set_fusion(self._h, FUSION[mode]), self)

    def set_batch_cfg(self, schedule: str | None = "phases", tile_h: int = 0):
        """Schedule ("phases" or "queue") and tile height of this context's
        batched launches; None restores the default."""
        if schedule is None:
            _check(lib().gf_ctx_set_batch_cfg(self._h, None), self)
        else:
            c = gf_batch_cfg(SCHEDULES[schedule], int(tile_h))
            _check(lib().gf_ctx_set_batch_cfg(self._h, ctypes.byref(c)), self)

    def set_wait_limit(self, polls: int | None = None):
        """Polls of the queue schedule's bounded waits before a tile gives up
        (None: the default of about three seconds)."""
        _check(lib().gf_ctx_set_wait_limit(self._h, -1 if polls is None else int(polls)), self)

    def tune_batched(self, Is, ps, prs, qs=None, workspace=None, reps: int = 3, stream=None):
        """Time every tile height of the phase schedule (of the queue
        schedule when the context is set to it) on this batch, keep the
        fastest for the context.  Returns (best dict, [(dict, ms), ...])."""
        if qs is None:
            qs = [_out_like(p, None) for p in ps]
        n = len(Is)
        aI, ap, aq, apr = _arrays(Is, ps, qs, prs)
        if workspace is None:
            workspace = _workspace(lib().gf_batched_workspace_bytes(n, aI, ap, apr), ps[0].device)
        best = gf_batch_cfg()
        res = (gf_batch_tune_result * 16)()
        cnt = ctypes.c_int32()
        _check(lib().gf_tune_batched(self._h, n, aI, ap, aq, apr, ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel() * workspace.element_size(), _stream(stream),
                                     int(reps), ctypes.byref(best), res, 16, ctypes.byref(cnt)), self)
        return best.as_dict(), [(res[i].cfg.as_dict(), res[i].ms) for i in range(cnt.value)]

    def gf_submit(self, I, p, q, r: int, s: int, eps: float, sub: str = "nearest", border: str = "clip") -> int:
        """Queue a request; returns its ticket.  I, p, q are kept alive here
        until gf_poll reports the request finished."""
        t = ctypes.c_uint64()
        _check(lib().gf_submit(self._h, ctypes.byref(image(I)), ctypes.byref(image(p)),
                               ctypes.byref(image(q)), ctypes.byref(params(r, s, eps, sub, border)),
                               ctypes.byref(t)), self)
        self._keep[t.value] = (I, p, q)
        return t.value

    def gf_poll(self, ticket: int, wait_ms: int = 0):
        """Returns (status, ReqStats or None); raises on a failed request."""
        st = gf_req_stats()
        rc = lib().gf_poll(self._h, ctypes.c_uint64(ticket), int(wait_ms), ctypes.byref(st))
        if rc == GF_PENDING or rc == GF_ETIMEDOUT:
            return rc, None
        self._keep.pop(ticket, None)
        _check(rc, self)
        return rc, ReqStats(st.t_submit, st.t_admit, st.t_start, st.t_done)
