"""Visibility-frequency crop volume of the evaluation protocol (CityGaussianV2 Sec. 4).

The visible frequency of every ground-truth point over all views, the threshold, the height range
and the ground-plane coordinates run in libcgv2r's kernels (``cgv2_visibility_count``,
``cgv2_crop_volume``); the alpha shape of the kept ground points runs on the host, as in the paper.

    cnt = visibility_count(points, cams, radius, filter_px)
    keep, ground, (h_min, h_max) = crop_volume(points, cnt, tau, T)
    area, boundary = alpha_shape(ground.cpu().numpy(), alpha)
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, ptr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def visibility_count(points, cams: Sequence, radius: float, filter_px: float, count=None, ws=None):
    """Visible frequency of points [3][m] (float32, device) over the views ``cams`` (generator cameras or
    a ctypes camera array): count [m] (int32-stored u32, += into ``count`` when given)."""
    L = _lib.lib()
    assert points.is_cuda and points.dtype == torch.float32 and points.is_contiguous() and points.shape[0] == 3
    m = points.shape[1]
    arr = cams if isinstance(cams, ctypes.Array) else _lib.camera_array(cams)
    V = len(arr)
    if count is None:
        count = torch.zeros(max(m, 1), dtype=torch.int32, device=points.device)[:m]
    need = max(L.cgv2_visibility_workspace(V), 256)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=points.device)
    check(L.cgv2_visibility_count(ptr(points), m, arr, V, float(radius), float(filter_px), ptr(count), ptr(ws),
                                  ws.numel(), _stream()), "cgv2_visibility_count")
    return count


def crop_volume(points, count, tau: int, T):
    """(keep [m] uint8, ground [2][kept] float64, (h_min, h_max)) of the points seen in >= tau views;
    T is the 3x4 ground transform.  Reads the kept count and the height range back (a synchronisation)."""
    L = _lib.lib()
    m = points.shape[1]
    dev = points.device
    Tm = np.ascontiguousarray(np.asarray(T, np.float64).reshape(12))
    keep = torch.empty(max(m, 1), dtype=torch.uint8, device=dev)
    ground = torch.empty((2, max(m, 1)), dtype=torch.float64, device=dev)
    hrange = torch.empty(2, dtype=torch.float64, device=dev)
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(L.cgv2_crop_workspace(m), 256), dtype=torch.uint8, device=dev)
    check(L.cgv2_crop_volume(ptr(points), m, ptr(count), int(tau), Tm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ptr(keep), ptr(ground), ptr(hrange), ptr(kept), ptr(ws), ws.numel(), _stream()),
          "cgv2_crop_volume")
    k = int(kept.item())
    h = hrange.cpu().numpy()
    return keep[:m], ground[:, :k] if m else ground[:, :0], (float(h[0]), float(h[1]))


def alpha_shape(xy, alpha: float):
    """Alpha shape of 2-D points xy [2][k] (host): the Delaunay triangles whose circumradius is below
    ``alpha`` (scene units).  Returns (area, boundary edges [e][2] as point indices).  alpha = inf gives
    the convex hull."""
    from scipy.spatial import Delaunay
    P = np.asarray(xy, np.float64).T
    if P.shape[0] < 3:
        return 0.0, np.zeros((0, 2), np.int64)
    tri = Delaunay(P)
    S = tri.simplices
    a, b, c = P[S[:, 0]], P[S[:, 1]], P[S[:, 2]]
    la = np.linalg.norm(b - c, axis=1)
    lb = np.linalg.norm(c - a, axis=1)
    lc = np.linalg.norm(a - b, axis=1)
    area2 = np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    with np.errstate(divide="ignore", invalid="ignore"):
        R = la * lb * lc / (2.0 * area2)
    sel = area2 > 0
    if np.isfinite(alpha):
        sel &= R < alpha
    S = S[sel]
    area = 0.5 * float(area2[sel].sum())
    # boundary: edges used by exactly one kept triangle
    e = np.sort(np.concatenate([S[:, [0, 1]], S[:, [1, 2]], S[:, [2, 0]]]), axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    return area, uniq[cnt == 1]
