"""Device-resident rasterizer engine over the C ABI, and its torch.autograd form.

PyTorch supplies device memory and the stream; every step runs in libcgv2r's kernels.

    eng = Engine(n, width, height, views=1, capacity=...)
    eng.project(params, cams); eng.bin_sort(cams); eng.render(cams)
    eng.loss(target); eng.backward(params, cams, grads); eng.densify(params, cams, state)

``Rasterize2DGS`` / ``L1SSIMLoss`` wrap the same calls as autograd Functions: the loss's backward
stores the SSIM-only image gradient on the engine, and the rasterizer's backward consumes it to
produce the decomposed densification gradient (CityGaussianV2 Eq. 2) next to the total one.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

import torch

from . import _lib
from ._lib import check, ptr

LAMBDA_SSIM = 0.2


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Params:
    """Surfel parameters on the device, float32: geometry planar ([3][n], [2][n], [4][n], [n]) and the SH
    coefficients as one block per surfel, sh[n][(deg+1)^2][3]."""

    def __init__(self, mean, log_scale, quat, opacity_logit, sh, sh_degree: int):
        self.mean, self.log_scale, self.quat = mean, log_scale, quat
        self.opacity_logit, self.sh, self.sh_degree = opacity_logit, sh, sh_degree
        for t in (mean, log_scale, quat, opacity_logit, sh):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        f = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return cls(f(scene.mean), f(scene.log_scale), f(scene.quat), f(scene.opacity_logit),
                   f(np.ascontiguousarray(scene.sh.transpose(2, 0, 1))), scene.sh_degree)

    @staticmethod
    def sh_planar(sh) -> np.ndarray:
        """[n][K][3] (this layout) -> [K][3][n] (the generators' and the oracle's layout)."""
        a = sh.detach().cpu().numpy() if isinstance(sh, torch.Tensor) else np.asarray(sh)
        return np.ascontiguousarray(a.transpose(1, 2, 0))

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def struct(self) -> _lib.Surfels:
        s = _lib.Surfels()
        s.n, s.sh_degree = self.n, self.sh_degree
        s.mean, s.log_scale, s.quat = ptr(self.mean), ptr(self.log_scale), ptr(self.quat)
        s.opacity_logit, s.sh = ptr(self.opacity_logit), ptr(self.sh)
        return s

    def zeros_like(self) -> "Params":
        return Params(*(torch.zeros_like(t) for t in (self.mean, self.log_scale, self.quat, self.opacity_logit,
                                                       self.sh)), self.sh_degree)


class Grads:
    """Parameter gradients (+=) and the per-view total / SSIM-only view-space gradients."""

    def __init__(self, params: Params, views: int):
        z = params.zeros_like()
        self.mean, self.log_scale, self.quat, self.opacity_logit, self.sh = (z.mean, z.log_scale, z.quat,
                                                                           z.opacity_logit, z.sh)
        n = params.n
        self.n, self.sh_degree = n, params.sh_degree
        dev = params.mean.device
        self.g_view_total = torch.zeros((views, 2, n), device=dev)
        self.g_view_ssim = torch.zeros((views, 2, n), device=dev)

    def zero_(self):
        """cgv2_zero_grads on the current stream (the parameter gradients; the view-space ones are
        overwritten by each backward)."""
        check(_lib.lib().cgv2_zero_grads(ctypes.byref(self.struct()), self.n, self.sh_degree, _stream()),
              "cgv2_zero_grads")

    def struct(self) -> _lib.Grads:
        g = _lib.Grads()
        g.d_mean, g.d_log_scale, g.d_quat = ptr(self.mean), ptr(self.log_scale), ptr(self.quat)
        g.d_opacity_logit, g.d_sh = ptr(self.opacity_logit), ptr(self.sh)
        g.g_view_total, g.g_view_ssim = ptr(self.g_view_total), ptr(self.g_view_ssim)
        return g


class DensifyState:
    def __init__(self, n: int, views: int = 1, device="cuda"):
        self.accum_dgd = torch.zeros(n, device=device)
        self.accum_total = torch.zeros(n, device=device)
        self.max_radius = torch.zeros(n, device=device)
        self.denom = torch.zeros(n, dtype=torch.int32, device=device)
        self.mask = torch.zeros(n, dtype=torch.uint8, device=device)
        self.counters = torch.zeros(8, dtype=torch.int32, device=device)
        self.scale = torch.zeros(max(views, 1), device=device)

    def reset(self):
        for t in (self.accum_dgd, self.accum_total, self.max_radius, self.denom, self.mask, self.counters):
            t.zero_()

    def struct(self) -> _lib.DensifyState:
        s = _lib.DensifyState()
        s.accum_dgd, s.accum_total, s.max_radius = ptr(self.accum_dgd), ptr(self.accum_total), ptr(self.max_radius)
        s.denom, s.mask, s.counters, s.scale = ptr(self.denom), ptr(self.mask), ptr(self.counters), ptr(self.scale)
        return s


class Engine:
    """Buffers for V views of one resolution and n surfels; each method is one C-ABI call."""

    def __init__(self, n: int, width: int, height: int, views: int = 1, capacity: Optional[int] = None,
                 device="cuda", backward: bool = True, images: bool = True):
        """images=False (render-only engines whose caller binds its own buffers, see bind_bins and
        bind_images): no image, checkpoint or bin buffers are allocated; bind them before rendering."""
        L = _lib.lib()
        self.n, self.W, self.H, self.V = int(n), int(width), int(height), int(views)
        self.tiles_x = (self.W + 15) // 16
        self.tiles_y = (self.H + 15) // 16
        self.tiles = self.tiles_x * self.tiles_y
        self.device = device
        V, H, W = self.V, self.H, self.W
        vn = max(V * n, 1)
        self.rec = torch.empty(vn * _lib.REC_FLOATS, device=device)
        self.rect = torch.empty(vn * 4, dtype=torch.int16, device=device)
        self.radius = torch.empty(vn, device=device)
        self.flags = torch.empty(vn, dtype=torch.uint8, device=device)
        self.visible = torch.empty(vn, dtype=torch.int32, device=device)
        self.visible_start = torch.zeros(V + 1, dtype=torch.int32, device=device)
        self.ranges = torch.zeros(V * self.tiles + 1, dtype=torch.int32, device=device)
        # render launch order (heaviest tiles first), written by each bin_sort
        self.order = torch.empty(max(V * self.tiles, 1), dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.needed = torch.zeros(1, dtype=torch.int64, device=device)
        if images:
            self.rgb = torch.empty((V, 3, H, W), device=device)
            self.depth = torch.empty((V, H, W), device=device)
            self.depth_med = torch.empty((V, H, W), device=device)
            self.normal = torch.empty((V, 3, H, W), device=device)
            self.alpha = torch.empty((V, H, W), device=device)
            self.T_final = torch.empty((V, H, W), device=device)
            self.last = torch.empty((V, H, W), dtype=torch.int32, device=device)
            self.med = torch.empty((V, H, W), dtype=torch.int32, device=device)
        else:
            self.rgb = self.depth = self.depth_med = self.normal = self.alpha = None
            self.T_final = self.last = self.med = None
        self.backward_enabled = backward and images
        if backward:
            self.d_img = torch.empty((V, 3, H, W), device=device)
            self.d_img_ssim = torch.empty((V, 3, H, W), device=device)
            self.loss_val = torch.zeros((V, 3), device=device)
            self.ws_loss = torch.empty(L.cgv2_loss_workspace(W, H, V), dtype=torch.uint8, device=device)
            self.ws_bwd = torch.empty(max(L.cgv2_render_bwd_workspace(n, V), 256), dtype=torch.uint8, device=device)
            self.ws_dens = torch.empty(max(L.cgv2_densify_workspace(n, V), 256), dtype=torch.uint8, device=device)
        self.pending_ssim = None
        # bumped by every call that rewrites the records, bins, images or checkpoint (generation) and by
        # every loss call (loss_generation): the autograd Functions check them so that a backward never
        # reads the state of a later forward
        self.generation = 0
        self.loss_generation = 0
        if images:
            self.set_capacity(capacity if capacity is not None else max(1 << 20, 16 * n * V))
        else:
            self.capacity, self.ids, self.ws_bin, self.qmask = 0, None, None, None
            self._bins = _lib.Bins(0, None, ptr(self.ranges), ptr(self.status), ptr(self.needed), ptr(self.order))
        self._proj = _lib.Proj(ptr(self.rec), ptr(self.rect), ptr(self.radius), ptr(self.flags), ptr(self.visible),
                               ptr(self.visible_start))
        self._img = _lib.Image(ptr(self.rgb), ptr(self.depth), ptr(self.depth_med), ptr(self.normal),
                               ptr(self.alpha), ptr(self.T_final), ptr(self.last), ptr(self.med), ptr(self.qmask))

    def set_capacity(self, capacity: int):
        L = _lib.lib()
        self.capacity = int(capacity)
        self.ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
        self.ws_bin = torch.empty(L.cgv2_bin_sort_workspace(self.capacity, self.V, self.tiles, self.n), dtype=torch.uint8,
                                  device=self.device)
        self._bins = _lib.Bins(self.capacity, ptr(self.ids), ptr(self.ranges), ptr(self.status), ptr(self.needed),
                               ptr(self.order))
        # per list entry quadrant-contribution mask written by the forward for the backward
        self.qmask = (torch.empty(max(self.capacity, 1), dtype=torch.uint8, device=self.device)
                      if self.backward_enabled else None)
        if hasattr(self, "_img"):
            self._img.qmask = ptr(self.qmask)

    def bind_bins(self, ids, ws, capacity: int):
        """Use caller-owned bins (no allocation): ids (>= capacity int32 entries) and a bin_sort workspace
        of at least cgv2_bin_sort_workspace(capacity, V, tiles, n) bytes for the calls that follow (the
        library checks it)."""
        assert ids.numel() >= max(capacity, 1)
        self.capacity, self.ids, self.ws_bin = int(capacity), ids, ws
        self._bins.capacity, self._bins.ids = self.capacity, ptr(ids)

    def bind_images(self, rgb=None, depth=None, normal=None, depth_med=None, alpha=None):
        """Render into caller-owned images ([V][c][h][w] for the call's resolution; None = not written).
        No checkpoint is kept: the engine then renders for serving only."""
        self._img = _lib.Image(ptr(rgb), ptr(depth), ptr(depth_med), ptr(normal), ptr(alpha), None, None, None, None)

    # ---- the five calls (+ loss) -------------------------------------------------------------
    def cams(self, cams: Sequence, exact: bool = True) -> ctypes.Array:
        """C camera array for a call.  exact=False admits any resolution up to the allocated one
        (all cameras of a call still share one size); outputs then occupy the leading elements."""
        assert len(cams) == self.V
        for c in cams:
            if exact:
                assert c.width == self.W and c.height == self.H
            else:
                assert c.width <= self.W and c.height <= self.H and c.width == cams[0].width \
                    and c.height == cams[0].height
        return _lib.camera_array(cams)

    def image(self, name: str, width: int, height: int):
        """The first view's output `name` for a call made at width x height (a view, no copy)."""
        t = getattr(self, name)
        per = {"rgb": 3, "normal": 3}.get(name, 1)
        flat = t.view(-1)[: per * width * height]
        return flat.view(per, height, width) if per > 1 else flat.view(height, width)

    def project(self, params, cams):
        """Projects a Params or a storage.CompactParams (serving storage) set."""
        self.generation += 1
        if getattr(params, "is_compact", False):
            check(_lib.lib().cgv2_project_compact(ctypes.byref(params.struct()), cams, self.V,
                                                  ctypes.byref(self._proj), _stream()), "cgv2_project_compact")
            return
        check(_lib.lib().cgv2_project(ctypes.byref(params.struct()), cams, self.V, ctypes.byref(self._proj),
                                      _stream()), "cgv2_project")

    def bin_sort(self, cams):
        self.generation += 1
        check(_lib.lib().cgv2_bin_sort(ctypes.byref(self._proj), cams, self.V, self.n, ctypes.byref(self._bins),
                                       ptr(self.ws_bin), self.ws_bin.numel(), _stream()), "cgv2_bin_sort")

    def render(self, cams):
        self.generation += 1
        check(_lib.lib().cgv2_render_fwd(ctypes.byref(self._proj), ctypes.byref(self._bins), cams, self.V, self.n,
                                         ctypes.byref(self._img), _stream()), "cgv2_render_fwd")

    def count(self, cams):
        """(evaluated, contributing, reverse-walked) pixel-entry pairs of the current bins."""
        c = torch.zeros(3, dtype=torch.int64, device=self.device)
        check(_lib.lib().cgv2_render_count(ctypes.byref(self._proj), ctypes.byref(self._bins), cams, self.V, self.n,
                                           ptr(c), _stream()), "cgv2_render_count")
        return [int(x) for x in c.cpu()]

    def loss(self, target, lam: float = LAMBDA_SSIM, img=None):
        img = self.rgb if img is None else img
        self.loss_generation += 1
        check(_lib.lib().cgv2_loss(ptr(img), ptr(target), self.V, self.W, self.H, lam, ptr(self.d_img),
                                   ptr(self.d_img_ssim), ptr(self.loss_val), ptr(self.ws_loss), self.ws_loss.numel(),
                                   _stream()), "cgv2_loss")
        return self.loss_val

    def backward(self, params: Params, cams, grads: Grads, d_rgb=None, d_depth=None, d_depth_med=None,
                 d_normal=None, d_alpha=None, d_rgb_ssim=None):
        if grads.g_view_total.shape[0] < self.V:
            raise ValueError("gradients hold fewer views than the engine")
        up = _lib.ImageGrad(ptr(d_rgb), ptr(d_depth), ptr(d_depth_med), ptr(d_normal), ptr(d_alpha),
                            ptr(d_rgb_ssim))
        check(_lib.lib().cgv2_render_bwd(ctypes.byref(params.struct()), ctypes.byref(self._proj),
                                         ctypes.byref(self._bins), cams, self.V, ctypes.byref(self._img),
                                         ctypes.byref(up), ctypes.byref(grads.struct()), ptr(self.ws_bwd),
                                         self.ws_bwd.numel(), _stream()), "cgv2_render_bwd")

    def backward_records(self, cams, d_rgb=None, d_depth=None, d_depth_med=None, d_normal=None, d_alpha=None,
                         d_rgb_ssim=None):
        """First stage of `backward`: pixel gradients -> record gradients (in this engine's workspace)."""
        up = _lib.ImageGrad(ptr(d_rgb), ptr(d_depth), ptr(d_depth_med), ptr(d_normal), ptr(d_alpha),
                            ptr(d_rgb_ssim))
        check(_lib.lib().cgv2_render_bwd_records(ctypes.byref(self._proj), ctypes.byref(self._bins), cams, self.V,
                                                 self.n, ctypes.byref(self._img), ctypes.byref(up), ptr(self.ws_bwd),
                                                 self.ws_bwd.numel(), _stream()), "cgv2_render_bwd_records")

    def project_backward(self, params: Params, cams, grads: Grads):
        """Second stage of `backward`: record gradients -> parameter and view-space gradients."""
        if grads.g_view_total.shape[0] < self.V:
            raise ValueError("gradients hold fewer views than the engine")
        check(_lib.lib().cgv2_project_bwd(ctypes.byref(params.struct()), ctypes.byref(self._proj), cams, self.V,
                                          ptr(self.ws_bwd), self.ws_bwd.numel(), ctypes.byref(grads.struct()),
                                          _stream()), "cgv2_project_bwd")

    def densify(self, params: Params, grads: Grads, state: DensifyState, omega=0.9, eta_min=0.05,
                grad_threshold=2e-4, no_alloc: bool = False):
        """cgv2_densify_stats; no_alloc=True calls cgv2_densify_stats_noalloc (the library's fixed per-GPU
        buffer instead of the engine's workspace)."""
        if state.scale.numel() < self.V or state.mask.numel() < self.n:
            raise ValueError("densify state holds fewer views or surfels than the engine")
        if grads.g_view_total.shape[0] < self.V:
            raise ValueError("gradients hold fewer views than the engine")
        prm = _lib.DensifyParams(omega, eta_min, grad_threshold)
        L = _lib.lib()
        if no_alloc:
            check(L.cgv2_densify_stats_noalloc(ctypes.byref(params.struct()), ctypes.byref(self._proj),
                                               ctypes.byref(grads.struct()), self.V, ctypes.byref(prm),
                                               ctypes.byref(state.struct()), _stream()), "cgv2_densify_stats_noalloc")
            return
        check(L.cgv2_densify_stats(ctypes.byref(params.struct()), ctypes.byref(self._proj),
                                   ctypes.byref(grads.struct()), self.V, ctypes.byref(prm),
                                   ctypes.byref(state.struct()), ptr(self.ws_dens), self.ws_dens.numel(),
                                   _stream()), "cgv2_densify_stats")

    # ---- contribution-based trimming (Sec. 3.3) --------------------------------------------------
    def contribution(self, cams, gamma: float = 0.5, c_view=None, c_sum=None, pixels=None):
        """Eq. 3 for the engine's V views from the current bins: c_view [V][n] (C per view), c_sum [n]
        (+= sum over the V views), pixels [V][n] (|P|, int32 storage of u32); any may be None."""
        L = _lib.lib()
        need = L.cgv2_contribution_workspace(self.n, self.V)
        if getattr(self, "ws_contrib", None) is None or self.ws_contrib.numel() < need:
            self.ws_contrib = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        check(L.cgv2_contribution(ctypes.byref(self._proj), ctypes.byref(self._bins), cams, self.V, self.n,
                                  float(gamma), ptr(c_view), ptr(c_sum), ptr(pixels), ptr(self.ws_contrib),
                                  self.ws_contrib.numel(), _stream()), "cgv2_contribution")

    # ---- helpers -------------------------------------------------------------------------------
    def overflowed(self) -> bool:
        return bool(self.status.item() != 0)

    def fit_capacity(self, params: Params, cams, slack: float = 1.25):
        """Project + bin once, read the intersection count and size the bins (synchronises)."""
        self.project(params, cams)
        self.status.zero_()
        self.bin_sort(cams)
        need = int(self.needed.item())
        if need > self.capacity or self.status.item() != 0:
            self.set_capacity(int(need * slack) + 1024)
            self.status.zero_()
        return need

    def forward(self, params: Params, cams):
        self.project(params, cams)
        self.bin_sort(cams)
        self.render(cams)


def trim_mask(c, ratio: float):
    """Sec. 3.3 trimming on a device array of contributions c [n] (float32, >= 0): returns
    (bound [1], mask [n] uint8, removed [1] int32-stored u32), all on the device, stream-ordered."""
    L = _lib.lib()
    n = c.numel()
    ws = torch.empty(max(L.cgv2_trim_workspace(n), 256), dtype=torch.uint8, device=c.device)
    bound = torch.empty(1, dtype=torch.float32, device=c.device)
    mask = torch.empty(n, dtype=torch.uint8, device=c.device)
    removed = torch.empty(1, dtype=torch.int32, device=c.device)
    check(L.cgv2_trim_mask(ptr(c), n, float(ratio), ptr(bound), ptr(mask), ptr(removed), ptr(ws), ws.numel(),
                           _stream()), "cgv2_trim_mask")
    return bound, mask, removed


class DensifyPlan:
    """Device outputs of cgv2_densify_plan: actions [n] (0 keep, 1 clone, 2 split, 3 remove), dst [2][n]
    (int32-stored u32 slots), counts [5] int64 (keep, clone, split, removed, output size)."""

    def __init__(self, actions, dst, counts):
        self.actions, self.dst, self.counts = actions, dst, counts

    def n_out(self) -> int:
        """Output size (reads the device count: a synchronisation)."""
        return int(self.counts[4].item())


def _action_params(dense_scale, min_opacity, split_shrink):
    prm = _lib.ActionParams()
    prm.dense_scale, prm.min_opacity, prm.split_shrink = float(dense_scale), float(min_opacity), float(split_shrink)
    return prm


def densify_plan(params: Params, mask, remove=None, dense_scale: float = 0.01, min_opacity: float = 0.005,
                 ws=None) -> DensifyPlan:
    """Per-surfel densification action (Sec. 3.2 candidates = bit 4 of ``mask``, Sec. 3.3 removal =
    ``remove``), stream-ordered; nothing is read back."""
    L = _lib.lib()
    n = params.n
    dev = params.mean.device
    actions = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    dst = torch.empty((2, max(n, 1)), dtype=torch.int32, device=dev)
    counts = torch.empty(5, dtype=torch.int64, device=dev)
    need = max(L.cgv2_densify_plan_workspace(n), 256)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    s = params.struct()
    check(L.cgv2_densify_plan(ctypes.byref(s), ptr(mask), ptr(remove),
                              ctypes.byref(_action_params(dense_scale, min_opacity, 1.6)), ptr(actions), ptr(dst),
                              ptr(counts), ptr(ws), ws.numel(), _stream()), "cgv2_densify_plan")
    return DensifyPlan(actions[:n], dst[:, :n] if n else dst[:, :0], counts)


def densify_apply(params: Params, plan: DensifyPlan, z, split_shrink: float = 1.6, n_out: Optional[int] = None,
                  out: Optional[Params] = None, src=None):
    """The new surfel set of a plan: (Params, src) with src [n_out] the slot -> (source << 2 | kind) map.
    z [n][2][2] float32 (device) are the children's standard-normal offsets.  n_out defaults to the
    plan's count (read from the device); out / src may be given (n_out surfels, n_out int32)."""
    L = _lib.lib()
    n = params.n
    if n_out is None:
        n_out = plan.n_out() if out is None else out.n
    dev = params.mean.device
    K = (params.sh_degree + 1) ** 2
    if out is None:
        out = Params(torch.empty((3, n_out), device=dev), torch.empty((2, n_out), device=dev),
                     torch.empty((4, n_out), device=dev), torch.empty(n_out, device=dev),
                     torch.empty((n_out, K, 3), device=dev), params.sh_degree)
    assert out.n == n_out and out.sh_degree == params.sh_degree
    if src is None:
        src = torch.empty(max(n_out, 1), dtype=torch.int32, device=dev)
    assert src.dtype == torch.int32 and src.numel() >= n_out
    if n:
        assert z.is_cuda and z.dtype == torch.float32 and z.is_contiguous() and z.numel() == 4 * n
    o = _lib.SurfelsOut()
    o.n, o.sh_degree = n_out, params.sh_degree
    o.mean, o.log_scale, o.quat = ptr(out.mean), ptr(out.log_scale), ptr(out.quat)
    o.opacity_logit, o.sh = ptr(out.opacity_logit), ptr(out.sh)
    s = params.struct()
    check(L.cgv2_densify_apply(ctypes.byref(s), ptr(plan.actions), ptr(plan.dst), ptr(plan.counts),
                               ptr(z) if n else None, ctypes.byref(_action_params(0.0, 0.0, split_shrink)),
                               ctypes.byref(o), ptr(src), _stream()), "cgv2_densify_apply")
    return out, src[:n_out]


def densify_gather(field, src, plan: DensifyPlan, n_out: int, blocked: bool = False, zero_new: bool = False):
    """Re-lays a per-surfel float32 field (planar [C][n] / [n], or blocked [n][C]) into the new set."""
    L = _lib.lib()
    assert field.is_cuda and field.dtype == torch.float32 and field.is_contiguous()
    if blocked:
        n, C = field.shape[0], int(field[0].numel()) if field.shape[0] else int(np.prod(field.shape[1:]))
        out = torch.empty((n_out,) + tuple(field.shape[1:]), dtype=torch.float32, device=field.device)
    else:
        n, C = field.shape[-1], int(np.prod(field.shape[:-1])) if field.dim() > 1 else 1
        out = torch.empty(tuple(field.shape[:-1]) + (n_out,), dtype=torch.float32, device=field.device)
    check(L.cgv2_densify_gather(ptr(field), n, C, 1 if blocked else 0, ptr(src), ptr(plan.counts),
                                1 if zero_new else 0, ptr(out), n_out, _stream()), "cgv2_densify_gather")
    return out


# ------------------------------------------------------------------------------------------------
# autograd form
# ------------------------------------------------------------------------------------------------

class Rasterize2DGS(torch.autograd.Function):
    """(mean, log_scale, quat, opacity_logit, sh) -> (rgb, depth, depth_med, normal, alpha) of V views.

    Saves nothing per fragment: the backward reads the engine's bins and the per-pixel
    checkpoint (T_final, last, med) written by the forward.  Gradients go to the parameters;
    the engine's ``grads`` also receives the total and SSIM-only view-space gradients.

    The outputs are the engine's own image buffers: they hold this forward's images until the engine's
    next forward.  A backward after another forward on the same engine raises (the checkpoint and bins it
    needs are gone), and so does a backward after an intersection overflow (the images are not valid;
    size the engine with ``fit_capacity`` and run again).
    """

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, sh, engine: Engine, cams, sh_degree: int):
        params = Params(mean.detach(), log_scale.detach(), quat.detach(), opacity_logit.detach(), sh.detach(),
                        sh_degree)
        engine.forward(params, cams)
        ctx.engine, ctx.cams, ctx.params = engine, cams, params
        ctx.generation = engine.generation
        # outputs the loss does not use reach the backward as None, not as zero images: the reverse
        # pass then skips the depth / normal / alpha terms entirely
        ctx.set_materialize_grads(False)
        return engine.rgb, engine.depth, engine.depth_med, engine.normal, engine.alpha

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_depth_med, d_normal, d_alpha):
        eng: Engine = ctx.engine
        p = ctx.params
        if eng.generation != ctx.generation:
            raise RuntimeError("Rasterize2DGS.backward: the engine ran another forward after this one; its bins "
                               "and checkpoint belong to that call (use one engine per pending graph)")
        if eng.overflowed():
            raise RuntimeError("Rasterize2DGS.backward: the intersection capacity overflowed in the forward "
                               f"(needed {int(eng.needed.item())}, capacity {eng.capacity}); the images are invalid")
        # fresh zeroed gradients (the ABI accumulates), handed to autograd without a copy
        g = Grads(p, eng.V)
        eng.grads = g
        c = lambda t: None if t is None else t.contiguous()
        # the SSIM-only image gradient, when the loss on this forward's images has left one
        pend = eng.pending_ssim
        d_ssim = pend[1] if pend is not None and pend[0] == ctx.generation else None
        eng.backward(p, ctx.cams, g, d_rgb=c(d_rgb), d_depth=c(d_depth), d_depth_med=c(d_depth_med),
                     d_normal=c(d_normal), d_alpha=c(d_alpha), d_rgb_ssim=d_ssim)
        eng.pending_ssim = None
        return g.mean, g.log_scale, g.quat, g.opacity_logit, g.sh, None, None, None


class L1SSIMLoss(torch.autograd.Function):
    """Per-view (1 - lambda) L1 + lambda (1 - SSIM), summed over views; its backward hands the
    SSIM-only image gradient to the engine for the decomposed densification gradient."""

    @staticmethod
    def forward(ctx, rgb, target, engine: Engine, lam: float):
        lv = engine.loss(target.contiguous(), lam, img=rgb.contiguous())
        ctx.engine = engine
        ctx.generation, ctx.loss_generation = engine.generation, engine.loss_generation
        return lv[:, 0].sum()

    @staticmethod
    def backward(ctx, g):
        eng: Engine = ctx.engine
        if eng.loss_generation != ctx.loss_generation:
            raise RuntimeError("L1SSIMLoss.backward: the engine ran another loss after this one; its image "
                               "gradients belong to that call")
        eng.pending_ssim = (ctx.generation, eng.d_img_ssim * g if not isinstance(g, float) else eng.d_img_ssim)
        return eng.d_img * g, None, None, None


def rasterize(params_t, engine: Engine, cams, sh_degree: int):
    return Rasterize2DGS.apply(*params_t, engine, cams, sh_degree)
