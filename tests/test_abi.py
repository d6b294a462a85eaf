"""The C ABI without a GPU: the library loads, exports every symbol the
header declares, and rejects invalid calls on the host before any HIP call.

Pointers below are fake device addresses: validation never dereferences
them, and every call here fails validation, so nothing is launched."""
import ctypes
import os
import re

import pytest

import gpuutil

gfp = gpuutil.ensure_built()
L = gfp.lib()
HEADER = os.path.join(gpuutil.ROOT, "include", "gf.h")


def test_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:gf_status|void|size_t|const char \*)\s*\*?\s*(gf_\w+)\s*\(",
                              text, re.M))
    assert declared == set(gfp.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def img(addr, c, h, w, dtype=gfp.GF_F32, rs=None, ps=None):
    rs = w if rs is None else rs
    ps = rs * h if ps is None else ps
    return gfp.gf_image(addr, dtype, c, h, w, rs, ps)


A_I, A_P, A_Q = 0x10000000, 0x20000000, 0x30000000


def call_fast(I, p, q, pr, ws=0x40000000, ws_bytes=1 << 40):
    return L.gf_fast(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), ctypes.byref(pr),
                     ctypes.c_void_p(ws), ws_bytes, None)


GOOD = dict(I=(A_I, 1, 64, 80), p=(A_P, 3, 64, 80), q=(A_Q, 3, 64, 80))


def good():
    return img(*GOOD["I"]), img(*GOOD["p"]), img(*GOOD["q"]), gfp.params(8, 4, 1e-2)


@pytest.mark.parametrize("case,status", [
    ("null_I_data", gfp.GF_EINVAL),
    ("negative_r", gfp.GF_EINVAL),
    ("zero_s", gfp.GF_EINVAL),
    ("zero_eps", gfp.GF_EINVAL),
    ("nan_eps", gfp.GF_EINVAL),
    ("inf_eps", gfp.GF_EINVAL),
    ("tiny_eps_underflows_fp32", gfp.GF_EINVAL),
    ("shape_mismatch", gfp.GF_EINVAL),
    ("channel_mismatch", gfp.GF_EINVAL),
    ("dtype_mismatch", gfp.GF_EINVAL),
    ("bad_dtype", gfp.GF_EINVAL),
    ("two_channel_guide", gfp.GF_ENOTSUP),
    ("colour_guide_radius_too_large", gfp.GF_ENOTSUP),
    ("row_stride_short", gfp.GF_EINVAL),
    ("plane_stride_short", gfp.GF_EINVAL),
    ("q_aliases_p", gfp.GF_EINVAL),
    ("q_overlaps_I_tail", gfp.GF_EINVAL),
    ("empty_image", gfp.GF_EINVAL),
    ("bad_border", gfp.GF_EINVAL),
    ("bad_subsample", gfp.GF_EINVAL),
    ("radius_too_large", gfp.GF_ENOTSUP),
    ("misaligned_data", gfp.GF_EINVAL),
    ("workspace_too_small", gfp.GF_ENOMEM),
    ("workspace_misaligned", gfp.GF_EINVAL),
])
def test_invalid_call_rejected_on_host(case, status):
    I, p, q, pr = good()
    ws, ws_bytes = 0x40000000, 1 << 40
    if case == "null_I_data":
        I.data = None
    elif case == "negative_r":
        pr.r = -1
    elif case == "zero_s":
        pr.s = 0
    elif case == "zero_eps":
        pr.eps = 0.0
    elif case == "nan_eps":
        pr.eps = float("nan")
    elif case == "inf_eps":
        pr.eps = float("inf")
    elif case == "tiny_eps_underflows_fp32":
        pr.eps = 1e-60
    elif case == "shape_mismatch":
        q = img(A_Q, 3, 64, 81)
    elif case == "channel_mismatch":
        q = img(A_Q, 2, 64, 80)
    elif case == "dtype_mismatch":
        p = img(A_P, 3, 64, 80, gfp.GF_F16)
    elif case == "bad_dtype":
        I.dtype = 7
    elif case == "two_channel_guide":
        I = img(A_I, 2, 64, 80)
    elif case == "colour_guide_radius_too_large":
        I = img(A_I, 3, 64, 80)
        pr.r, pr.s = 120, 4  # r' = 30: the colour coefficient tiles do not fit in LDS
    elif case == "row_stride_short":
        p = img(A_P, 3, 64, 80, rs=79)
    elif case == "plane_stride_short":
        p = img(A_P, 3, 64, 80, ps=64 * 80 - 1)
    elif case == "q_aliases_p":
        q = img(A_P, 3, 64, 80)
    elif case == "q_overlaps_I_tail":
        q = img(A_I + 4 * (64 * 80 - 1), 3, 64, 80)
    elif case == "empty_image":
        I, p, q = img(A_I, 1, 0, 80), img(A_P, 3, 0, 80), img(A_Q, 3, 0, 80)
    elif case == "bad_border":
        pr.border = 3
    elif case == "bad_subsample":
        pr.sub = 9
    elif case == "radius_too_large":
        pr.r, pr.s = 4000, 1
    elif case == "misaligned_data":
        I.data = A_I + 2
    elif case == "workspace_too_small":
        ws_bytes = 1024
    elif case == "workspace_misaligned":
        ws = 0x40000010
    assert call_fast(I, p, q, pr, ws, ws_bytes) == status
    assert gfp.last_error() != ""


def test_plain_validates_like_fast():
    I, p, q, _ = good()
    st = L.gf_plain(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), 4, -1.0,
                    gfp.GF_BORDER_CLIP, ctypes.c_void_p(0x40000000), 1 << 40, None)
    assert st == gfp.GF_EINVAL and "eps" in gfp.last_error()


def test_no_workspace_and_no_context_rejected():
    I, p, q, pr = good()
    assert L.gf_fast(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), ctypes.byref(pr),
                     None, 0, None) == gfp.GF_EINVAL


def test_request_interface_needs_context():
    I, p, q, pr = good()
    t = ctypes.c_uint64()
    assert L.gf_submit(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), ctypes.byref(pr),
                       ctypes.byref(t)) == gfp.GF_EINVAL
    assert L.gf_poll(None, 1, 0, None) == gfp.GF_EINVAL


def test_workspace_bytes():
    # 4C FP32 planes of ceil(h/s) rows, rows padded to 16 floats, planes to 64 floats
    pr = gfp.params(16, 4, 1e-3)
    hl, wl = 750, 1000
    lrs = -(-wl // 16) * 16
    lps = -(-(hl * lrs) // 64) * 64
    assert L.gf_workspace_bytes(3000, 4000, 3, ctypes.byref(pr)) == 4 * 3 * lps * 4
    assert L.gf_workspace_bytes(0, 4000, 3, ctypes.byref(pr)) == 0
    pr1 = gfp.params(16, 1, 1e-3)
    assert L.gf_workspace_bytes(10, 10, 1, ctypes.byref(pr1)) == 4 * 1 * 192 * 4
    # area subsampling adds I' and the C channels of p' (1 + C planes); borders add nothing
    pra = gfp.params(16, 4, 1e-3, "area")
    assert L.gf_workspace_bytes(3000, 4000, 3, ctypes.byref(pra)) == (4 * 3 + 1 + 3) * lps * 4
    prb = gfp.params(16, 4, 1e-3, "nearest", "reflect101")
    assert L.gf_workspace_bytes(3000, 4000, 3, ctypes.byref(prb)) == 4 * 3 * lps * 4
    pra1 = gfp.params(16, 1, 1e-3, "area")  # s = 1: the area mean of one pixel is that pixel, no pass
    assert L.gf_workspace_bytes(10, 10, 1, ctypes.byref(pra1)) == 4 * 1 * 192 * 4
    # a colour guide: a_0, a_1, a_2, b and their box means (8C planes), plus 3 + C with area subsampling
    assert L.gf_workspace_bytes_guide(3000, 4000, 3, 3, ctypes.byref(pr)) == 8 * 3 * lps * 4
    assert L.gf_workspace_bytes_guide(3000, 4000, 3, 3, ctypes.byref(pra)) == (8 * 3 + 3 + 3) * lps * 4
    assert L.gf_workspace_bytes_guide(3000, 4000, 1, 3, ctypes.byref(pr)) == L.gf_workspace_bytes(3000, 4000, 3, ctypes.byref(pr))
    assert L.gf_workspace_bytes_guide(3000, 4000, 2, 3, ctypes.byref(pr)) == 0


def test_prepared_batch_rejected_on_host():
    I, p, q, pr = good()
    n = 1
    aI, ap, aq, apr = ((gfp.gf_image * 1)(I), (gfp.gf_image * 1)(p), (gfp.gf_image * 1)(q),
                       (gfp.gf_params * 1)(pr))
    h = ctypes.c_void_p()

    def create(ws=0x40000000, ws_bytes=1 << 40, out=True, prs=apr):
        return L.gf_batch_create(None, n, aI, ap, aq, prs, ctypes.c_void_p(ws), ws_bytes, None,
                                 ctypes.byref(h) if out else None)

    assert create(out=False) == gfp.GF_EINVAL
    assert create(ws=0) == gfp.GF_EINVAL and "workspace" in gfp.last_error()
    assert create(ws=0x40000010) == gfp.GF_EINVAL
    assert create(ws_bytes=4096) == gfp.GF_ENOMEM and h.value is None
    bad = (gfp.gf_params * 1)(gfp.params(8, 4, 1e-2))
    bad[0].eps = 0.0
    assert create(prs=bad) == gfp.GF_EINVAL and h.value is None
    assert L.gf_batch_launch(None, None) == gfp.GF_EINVAL
    L.gf_batch_destroy(None)


def test_batch_cfg_needs_context():
    c = gfp.gf_batch_cfg(gfp.GF_BATCH_PHASES, 16)
    assert L.gf_ctx_set_batch_cfg(None, ctypes.byref(c)) == gfp.GF_EINVAL
    n = ctypes.c_int32(-1)
    assert L.gf_tune_batched(None, 1, None, None, None, None, None, 0, None, 1, None, None, 0,
                             ctypes.byref(n)) == gfp.GF_EINVAL


def test_footprint_bytes():
    # control words and descriptor table (256-byte granules) + a, b and their means (4C planes)
    pr = gfp.params(16, 4, 1e-3)
    hl, wl = 750, 1000
    lrs = -(-wl // 16) * 16
    lps = -(-(hl * lrs) // 64) * 64
    planes = 2 * (-(-(4 * lps * 2 * 3) // 256) * 256)
    fp = L.gf_footprint_bytes(3000, 4000, 3, gfp.GF_F16, ctypes.byref(pr))
    assert planes < fp <= planes + 256 + 256 * 4
    assert fp == L.gf_footprint_bytes(3000, 4000, 3, gfp.GF_F32, ctypes.byref(pr))
    assert L.gf_footprint_bytes(0, 4000, 3, gfp.GF_F32, ctypes.byref(pr)) == 0
    assert L.gf_footprint_bytes(30, 40, 3, 9, ctypes.byref(pr)) == 0


def test_joint_upsample_shapes_checked_on_host():
    # p_low must be ceil(h/s) x ceil(w/s); q full resolution
    I = img(A_I, 1, 64, 80)
    q = img(A_Q, 3, 64, 80)
    pr = gfp.params(8, 4, 1e-2)

    def call(p, q=q, pr=pr):
        return L.gf_joint_upsample(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), ctypes.byref(pr),
                                   ctypes.c_void_p(0x40000000), 1024, None)
    assert call(img(A_P, 3, 64, 80)) == gfp.GF_EINVAL          # full-resolution p
    assert call(img(A_P, 3, 16, 21)) == gfp.GF_EINVAL          # wrong low-res width
    assert call(img(A_P, 3, 16, 20), q=img(A_Q, 3, 16, 20)) == gfp.GF_EINVAL  # low-res q
    bad = gfp.params(8, 0, 1e-2)
    assert call(img(A_P, 3, 16, 20), pr=bad) == gfp.GF_EINVAL  # s = 0
    # right shapes: validation passes, the tiny workspace is then refused
    assert call(img(A_P, 3, 16, 20)) == gfp.GF_ENOMEM


def test_noalloc_host_checks():
    """gf_fast_noalloc validates like gf_fast and refuses, before any HIP
    call, a problem whose low-res maps exceed its fixed device array; the
    binding's size is the header's."""
    text = open(HEADER).read()
    m = re.search(r"#define GF_NOALLOC_MAX_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == gfp.NOALLOC_MAX_BYTES
    I, p, q, pr = good()
    bad = gfp.params(8, 4, 0.0)
    assert L.gf_fast_noalloc(None, ctypes.byref(I), ctypes.byref(p), ctypes.byref(q), ctypes.byref(bad),
                             None) == gfp.GF_EINVAL
    h, w = 4096, 4096  # 12 FP32 maps of 16 MP at s = 1
    big = [img(A_I, 1, h, w), img(A_P, 3, h, w), img(A_Q, 3, h, w)]
    pr1 = gfp.params(8, 1, 1e-3)
    assert L.gf_workspace_bytes(h, w, 3, ctypes.byref(pr1)) > gfp.NOALLOC_MAX_BYTES
    assert L.gf_fast_noalloc(None, *[ctypes.byref(x) for x in big], ctypes.byref(pr1), None) == gfp.GF_ENOMEM
    assert "scratch" in gfp.last_error()


def test_fusion_mode_needs_context():
    assert L.gf_ctx_set_fusion(None, gfp.GF_FUSE_ON) == gfp.GF_EINVAL
    assert "context" in gfp.last_error()
