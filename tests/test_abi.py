"""The C-ABI library: loads, exports every entry point of include/cgv2r.h, validates arguments and
sizes workspaces without touching a GPU (every case here returns before any HIP call)."""
import ctypes
import os
import re

import pytest

from paper_2411_00771_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgv2r.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cgv2_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_header_constants_match_binding():
    txt = open(HEADER).read()
    assert re.search(r"#define CGV2_REC_FLOATS (\d+)", txt).group(1) == str(_lib.REC_FLOATS)
    assert re.search(r"#define CGV2_TILE (\d+)", txt).group(1) == str(_lib.TILE)
    assert ctypes.sizeof(_lib.Camera) == 4 * (2 + 4 + 9 + 3 + 1 + 3)


def test_strerror_and_workspace_sizes():
    L = _lib.lib()
    assert L.cgv2_strerror(0) == b"ok" and L.cgv2_strerror(-2) == b"workspace too small"
    a = L.cgv2_bin_sort_workspace(1 << 20, 1, 6700, 1000)
    b = L.cgv2_bin_sort_workspace(1 << 21, 1, 6700, 1000)
    assert b - a >= 20 * (1 << 20)  # two u64 and one u32 array per intersection
    assert L.cgv2_bin_sort_workspace(1 << 20, 1, 6700, 10 ** 6) >= a + 4 * (10 ** 6 - 1000)
    assert L.cgv2_bin_sort_workspace(-1, 1, 10, 5) == 0 and L.cgv2_bin_sort_workspace(10, 0, 10, 5) == 0
    assert L.cgv2_render_bwd_workspace(1000, 2) >= 19 * 4 * 1000 * 2
    assert L.cgv2_render_bwd_workspace(-1, 2) == 0 and L.cgv2_render_bwd_workspace(10, 0) == 0
    assert L.cgv2_loss_workspace(0, 10, 1) == 0
    assert L.cgv2_densify_workspace(10, 1) > 0
    # plan workspace: 24 bytes per workgroup of 2048 surfels, 256-byte aligned parts
    assert L.cgv2_densify_plan_workspace(0) > 0 and L.cgv2_densify_plan_workspace(-1) == 0
    assert L.cgv2_densify_plan_workspace(10 ** 7) >= 24 * (10 ** 7 // 2048)
    # visibility: one FP64 camera table row per view; crop: 20 bytes per workgroup of 2048 points
    assert L.cgv2_visibility_workspace(958) >= 958 * 56 * 8 and L.cgv2_visibility_workspace(0) == 0
    assert L.cgv2_crop_workspace(10 ** 7) >= 20 * (10 ** 7 // 2048) and L.cgv2_crop_workspace(-1) == 0


def _fake_proj():
    return _lib.Proj(*[ctypes.c_void_p(256 * (k + 1)) for k in range(6)])


def test_argument_validation_returns_einval():
    L = _lib.lib()
    cam = _lib.Camera()
    cam.width, cam.height = 64, 64
    cams = (_lib.Camera * 2)(cam, cam)
    s = _lib.Surfels(10, 3, *[ctypes.c_void_p(256)] * 5)
    p = _fake_proj()
    EINVAL = _lib.CGV2_EINVAL
    assert L.cgv2_project(None, cams, 1, ctypes.byref(p), None) == EINVAL
    assert L.cgv2_project(ctypes.byref(s), cams, 0, ctypes.byref(p), None) == EINVAL
    bad = _lib.Surfels(10, 4, *[ctypes.c_void_p(256)] * 5)
    assert L.cgv2_project(ctypes.byref(bad), cams, 1, ctypes.byref(p), None) == EINVAL
    neg = _lib.Surfels(-1, 3, *[ctypes.c_void_p(256)] * 5)
    assert L.cgv2_project(ctypes.byref(neg), cams, 1, ctypes.byref(p), None) == EINVAL
    nul = _lib.Surfels(10, 3, None, None, None, None, None)
    assert L.cgv2_project(ctypes.byref(nul), cams, 1, ctypes.byref(p), None) == EINVAL
    other = _lib.Camera()
    other.width, other.height = 32, 64
    mixed = (_lib.Camera * 2)(cam, other)
    assert L.cgv2_project(ctypes.byref(s), mixed, 2, ctypes.byref(p), None) == EINVAL
    zero = _lib.Camera()
    assert L.cgv2_project(ctypes.byref(s), ctypes.byref(zero), 1, ctypes.byref(p), None) == EINVAL
    huge = _lib.Camera()
    huge.width, huge.height = 16 * 70000, 16
    assert L.cgv2_project(ctypes.byref(s), ctypes.byref(huge), 1, ctypes.byref(p), None) == EINVAL
    bins = _lib.Bins(100, ctypes.c_void_p(256), None, ctypes.c_void_p(256), ctypes.c_void_p(256))
    assert L.cgv2_bin_sort(ctypes.byref(p), cams, 1, 10, ctypes.byref(bins), ctypes.c_void_p(256), 1 << 30,
                           None) == EINVAL
    img = _lib.Image()
    assert L.cgv2_render_fwd(ctypes.byref(p), None, cams, 1, 10, ctypes.byref(img), None) == EINVAL
    assert L.cgv2_loss(None, None, 1, 8, 8, 0.2, None, None, None, None, 0, None) == EINVAL
    g = _lib.Grads()
    up = _lib.ImageGrad()
    okbins = _lib.Bins(100, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256))
    # backward without the forward checkpoint
    assert L.cgv2_render_bwd(ctypes.byref(s), ctypes.byref(p), ctypes.byref(okbins), cams, 1, ctypes.byref(img),
                             ctypes.byref(up), ctypes.byref(g), ctypes.c_void_p(256), 1 << 30, None) == EINVAL
    assert L.cgv2_render_bwd_records(ctypes.byref(p), ctypes.byref(okbins), cams, 1, 10, ctypes.byref(img),
                                     ctypes.byref(up), ctypes.c_void_p(256), 1 << 30, None) == EINVAL
    # zeroing: no gradients, a missing or misaligned array, n < 0, an SH degree outside 0-3
    assert L.cgv2_zero_grads(None, 10, 3, None) == EINVAL
    assert L.cgv2_zero_grads(ctypes.byref(g), 10, 3, None) == EINVAL
    ga = _lib.Grads(*[ctypes.c_void_p(256 * (k + 1)) for k in range(7)])
    assert L.cgv2_zero_grads(ctypes.byref(ga), -1, 3, None) == EINVAL
    assert L.cgv2_zero_grads(ctypes.byref(ga), 10, 4, None) == EINVAL
    gm = _lib.Grads(*([ctypes.c_void_p(256 * (k + 1)) for k in range(4)] + [ctypes.c_void_p(258)] +
                      [ctypes.c_void_p(256)] * 2))
    assert L.cgv2_zero_grads(ctypes.byref(gm), 10, 3, None) == EINVAL
    # parameter gradients missing
    assert L.cgv2_project_bwd(ctypes.byref(s), ctypes.byref(p), cams, 1, ctypes.c_void_p(256), 1 << 30,
                              ctypes.byref(g), None) == EINVAL
    assert L.cgv2_project_bwd(ctypes.byref(s), ctypes.byref(p), cams, 1, ctypes.c_void_p(256), 1 << 30, None,
                              None) == EINVAL
    # contribution: bad gamma, missing bins; trim: bad ratio, n < 1, missing mask
    ws = ctypes.c_void_p(256)
    assert L.cgv2_contribution(ctypes.byref(p), ctypes.byref(okbins), cams, 1, 10, 1.5, None, None, None, ws,
                               1 << 30, None) == EINVAL
    assert L.cgv2_contribution(ctypes.byref(p), None, cams, 1, 10, 0.5, None, None, None, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_trim_mask(ws, 10, 1.5, None, ws, None, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_trim_mask(ws, 0, 0.1, None, ws, None, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_trim_mask(ws, 10, 0.1, None, None, None, ws, 1 << 30, None) == EINVAL
    # densification action: n beyond 2^30, missing outputs, bad thresholds, mismatched output degree
    ap = _lib.ActionParams(0.01, 0.005, 1.6)
    big = _lib.Surfels(1 << 30, 3, *[ctypes.c_void_p(256)] * 5)
    assert L.cgv2_densify_plan(ctypes.byref(big), ws, None, ctypes.byref(ap), ws, ws, ws, ws, 1 << 40,
                               None) == EINVAL
    assert L.cgv2_densify_plan(ctypes.byref(s), ws, None, ctypes.byref(ap), None, ws, ws, ws, 1 << 30,
                               None) == EINVAL
    assert L.cgv2_densify_plan(ctypes.byref(s), ws, None, ctypes.byref(_lib.ActionParams(0.01, 1.5, 1.6)), ws, ws,
                               ws, ws, 1 << 30, None) == EINVAL
    so = _lib.SurfelsOut(20, 3, *[ctypes.c_void_p(256)] * 5)
    assert L.cgv2_densify_apply(ctypes.byref(s), ws, ws, ws, ws, ctypes.byref(_lib.ActionParams(0.01, 0.0, 0.0)),
                                ctypes.byref(so), ws, None) == EINVAL
    so2 = _lib.SurfelsOut(20, 2, *[ctypes.c_void_p(256)] * 5)
    assert L.cgv2_densify_apply(ctypes.byref(s), ws, ws, ws, ws, ctypes.byref(ap), ctypes.byref(so2), ws,
                                None) == EINVAL
    assert L.cgv2_densify_apply(ctypes.byref(s), ws, ws, ws, ws, ctypes.byref(ap), ctypes.byref(so), None,
                                None) == EINVAL
    assert L.cgv2_densify_gather(ws, 10, 0, 0, ws, ws, 0, ws, 20, None) == EINVAL
    assert L.cgv2_densify_gather(ws, 10, 3, 2, ws, ws, 0, ws, 20, None) == EINVAL
    assert L.cgv2_densify_gather(None, 10, 3, 0, ws, ws, 0, ws, 20, None) == EINVAL
    # visibility: V < 1, negative radius, a camera without znear; crop: missing transform or outputs
    vc = _lib.Camera()
    vc.width, vc.height, vc.fx, vc.fy, vc.znear = 64, 48, 50.0, 50.0, 0.2
    assert L.cgv2_visibility_count(ws, 10, ctypes.byref(vc), 0, 0.1, 1.0, ws, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_visibility_count(ws, 10, ctypes.byref(vc), 1, -0.1, 1.0, ws, ws, 1 << 30, None) == EINVAL
    bad_near = _lib.Camera()
    bad_near.width, bad_near.height, bad_near.fx, bad_near.fy = 64, 48, 50.0, 50.0
    assert L.cgv2_visibility_count(ws, 10, ctypes.byref(bad_near), 1, 0.1, 1.0, ws, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_visibility_count(ws, 10, ctypes.byref(vc), 1, 0.1, 1.0, None, ws, 1 << 30, None) == EINVAL
    T = (ctypes.c_double * 12)()
    assert L.cgv2_crop_volume(ws, 10, ws, 1, None, ws, ws, ws, ws, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_crop_volume(ws, 10, ws, 1, T, None, ws, ws, ws, ws, 1 << 30, None) == EINVAL
    assert L.cgv2_crop_volume(ws, -1, ws, 1, T, ws, ws, ws, ws, ws, 1 << 30, None) == EINVAL
    prm = _lib.DensifyParams(0.9, 0.05, 2e-4)
    st = _lib.DensifyState()
    assert L.cgv2_densify_stats(ctypes.byref(s), ctypes.byref(p), ctypes.byref(g), 1, ctypes.byref(prm),
                                ctypes.byref(st), ctypes.c_void_p(256), 1 << 30, None) == EINVAL


def test_small_workspace_returns_eworkspace():
    L = _lib.lib()
    cam = _lib.Camera()
    cam.width, cam.height = 64, 64
    p = _fake_proj()
    bins = _lib.Bins(1000, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256))
    need = L.cgv2_bin_sort_workspace(1000, 1, 16, 10)
    assert L.cgv2_bin_sort(ctypes.byref(p), ctypes.byref(cam), 1, 10, ctypes.byref(bins), ctypes.c_void_p(256),
                           need - 1, None) == _lib.CGV2_EWORKSPACE
    v = ctypes.c_void_p(256)
    img = _lib.Image(*[v] * 8)
    up = _lib.ImageGrad()
    ws = L.cgv2_render_bwd_workspace(10, 1)
    assert L.cgv2_render_bwd_records(ctypes.byref(p), ctypes.byref(bins), ctypes.byref(cam), 1, 10, ctypes.byref(img),
                                     ctypes.byref(up), v, ws - 1, None) == _lib.CGV2_EWORKSPACE
    s = _lib.Surfels(10, 3, *[v] * 5)
    g = _lib.Grads(*[v] * 7)
    assert L.cgv2_project_bwd(ctypes.byref(s), ctypes.byref(p), ctypes.byref(cam), 1, v, ws - 1, ctypes.byref(g),
                              None) == _lib.CGV2_EWORKSPACE
    assert L.cgv2_contribution(ctypes.byref(p), ctypes.byref(bins), ctypes.byref(cam), 1, 10, 0.5, None, None, None, v,
                               L.cgv2_contribution_workspace(10, 1) - 1, None) == _lib.CGV2_EWORKSPACE
    assert L.cgv2_trim_mask(v, 1000, 0.1, None, v, None, v, L.cgv2_trim_workspace(1000) - 1,
                            None) == _lib.CGV2_EWORKSPACE
    assert L.cgv2_loss(v, v, 1, 64, 64, 0.2, v, v, v, v, L.cgv2_loss_workspace(64, 64, 1) - 1,
                       None) == _lib.CGV2_EWORKSPACE
    ap = _lib.ActionParams(0.01, 0.005, 1.6)
    assert L.cgv2_densify_plan(ctypes.byref(s), v, None, ctypes.byref(ap), v, v, v, v,
                               L.cgv2_densify_plan_workspace(10) - 1, None) == _lib.CGV2_EWORKSPACE
    vc = _lib.Camera()
    vc.width, vc.height, vc.fx, vc.fy, vc.znear = 64, 48, 50.0, 50.0, 0.2
    assert L.cgv2_visibility_count(v, 10, ctypes.byref(vc), 1, 0.1, 1.0, v, v, L.cgv2_visibility_workspace(1) - 1,
                                   None) == _lib.CGV2_EWORKSPACE
    T = (ctypes.c_double * 12)()
    assert L.cgv2_crop_volume(v, 5000, v, 1, T, v, v, v, v, v, L.cgv2_crop_workspace(5000) - 1,
                              None) == _lib.CGV2_EWORKSPACE


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.Cgv2Error):
        _lib.lib()


def test_no_gfx950_device_returns_eunsupported():
    """Valid arguments with no usable gfx950 device (this host has no GPU): every compute entry point
    returns CGV2_EUNSUPPORTED before launching anything, after its argument checks."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    L = _lib.lib()
    cam = _lib.Camera()
    cam.width, cam.height, cam.fx, cam.fy = 64, 48, 50.0, 50.0
    cams = (_lib.Camera * 1)(cam)
    s = _lib.Surfels(10, 3, *[ctypes.c_void_p(256)] * 5)
    p = _fake_proj()
    assert L.cgv2_project(ctypes.byref(s), cams, 1, ctypes.byref(p), None) == _lib.CGV2_EUNSUPPORTED
    # argument errors still come first
    assert L.cgv2_project(ctypes.byref(s), cams, 0, ctypes.byref(p), None) == _lib.CGV2_EINVAL
    b = _lib.Bins(1024, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), ctypes.c_void_p(1024), None)
    ws = L.cgv2_bin_sort_workspace(1024, 1, 12, 10)
    assert L.cgv2_bin_sort(ctypes.byref(p), cams, 1, 10, ctypes.byref(b), ctypes.c_void_p(4096), ctypes.c_size_t(ws),
                           None) == _lib.CGV2_EUNSUPPORTED
    lw = L.cgv2_loss_workspace(64, 48, 1)
    assert L.cgv2_loss(*[ctypes.c_void_p(256)] * 2, 1, 64, 48, ctypes.c_float(0.2), *[ctypes.c_void_p(256)] * 4,
                       ctypes.c_size_t(lw), None) == _lib.CGV2_EUNSUPPORTED
    assert L.cgv2_strerror(_lib.CGV2_EUNSUPPORTED) == b"unsupported device"
