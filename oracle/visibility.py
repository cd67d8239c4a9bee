"""FP64 reference of the visibility-frequency crop-volume estimate -- TEST INFRASTRUCTURE ONLY.

Sec. 4 (crop volume of the evaluation protocol): every ground-truth point is treated as a small
Gaussian primitive, all views are traversed and each point's number of views with a non-empty
visible mask is counted; points seen less often than a threshold are dropped, the height range of the
rest is taken and the rest is projected to the ground plane for an alpha shape.

Readings (the paper names the procedure, not its geometry; parity unpinned beyond the mathematics):
  * a point's primitive is an isotropic Gaussian whose footprint is the image of the sphere of radius
    rho around it (the extent a GS rasterizer gives an isotropic Gaussian), hulled with a disc of
    filter_px pixels around the projected centre (the screen low-pass filter);
  * its visible mask in a view is the rasterizer's: centre depth beyond znear and at least one pixel
    sample (i + 0.5, j + 0.5) inside the footprint's bounding box (no occlusion test);
  * a sphere reaching the camera plane (depth <= rho) has an unbounded image: visible;
  * height and ground coordinates are the third and first two coordinates of T p, with T the 3x4
    ground transform.

Plain numpy in float64; camera values are the float32 ones the device receives.
"""
from __future__ import annotations

import numpy as np

# relative distance to a decision threshold below which an FP64 evaluation in another order may
# decide differently
FRAGILE = 1e-9


def _cam(cam):
    a = cam.as_array()
    W, H = int(a[0]), int(a[1])
    fx, fy, cx, cy = a[2:6]
    R = a[6:15].reshape(3, 3)
    t = a[15:18]
    znear = a[18]
    return W, H, fx, fy, cx, cy, R, t, znear


def sphere_image_bbox(X, Y, Z, rho, fx, fy, cx, cy):
    """Bounding box of the image of the sphere of radius rho centred at camera-frame (X, Y, Z), Z > rho.

    The x extent is bounded by the two planes through the camera centre that contain its y axis and
    touch the sphere: in the xz plane these are the tangent lines from the origin to the circle of
    radius rho about (X, Z), whose slopes x/z are (X Z +- rho sqrt(X^2 + Z^2 - rho^2)) / (Z^2 - rho^2).
    Likewise for y."""
    den = Z * Z - rho * rho
    sx = np.sqrt(X * X + Z * Z - rho * rho)
    sy = np.sqrt(Y * Y + Z * Z - rho * rho)
    u0 = fx * ((X * Z - rho * sx) / den) + cx
    u1 = fx * ((X * Z + rho * sx) / den) + cx
    v0 = fy * ((Y * Z - rho * sy) / den) + cy
    v1 = fy * ((Y * Z + rho * sy) / den) + cy
    return u0, u1, v0, v1


def _near_int(x):
    return np.abs(x - np.round(x)) / np.maximum(1.0, np.abs(x))


def visible(points, cam, rho, filter_px):
    """(visible [m] bool, fragile [m] bool) of points [3][m] in one view."""
    W, H, fx, fy, cx, cy, R, t, znear = _cam(cam)
    P = np.asarray(points, np.float32).astype(np.float64)
    Xc = R @ P + t[:, None]
    X, Y, Z = Xc
    rho = float(np.float32(rho))
    rf = float(np.float32(filter_px))
    front = Z > znear
    reach = Z <= rho  # the sphere reaches the camera plane: unbounded image
    with np.errstate(divide="ignore", invalid="ignore"):
        u0, u1, v0, v1 = sphere_image_bbox(X, Y, Z, rho, fx, fy, cx, cy)
        uc, vc = fx * (X / Z) + cx, fy * (Y / Z) + cy
    ulo, uhi = np.minimum(u0, uc - rf), np.maximum(u1, uc + rf)
    vlo, vhi = np.minimum(v0, vc - rf), np.maximum(v1, vc + rf)
    with np.errstate(invalid="ignore"):
        i0 = np.maximum(0, np.ceil(ulo - 0.5))
        i1 = np.minimum(W - 1, np.floor(uhi - 0.5))
        j0 = np.maximum(0, np.ceil(vlo - 0.5))
        j1 = np.minimum(H - 1, np.floor(vhi - 0.5))
    vis = front & (reach | ((i0 <= i1) & (j0 <= j1)))
    # margins of the decisions: depth vs znear and vs rho, the four rect edges
    with np.errstate(invalid="ignore", divide="ignore"):
        m = np.abs(Z - znear) / np.maximum(1.0, np.abs(Z))
        m = np.minimum(m, np.abs(Z - rho) / np.maximum(1.0, np.abs(Z)))
        for e in (ulo - 0.5, uhi - 0.5, vlo - 0.5, vhi - 0.5):
            m = np.minimum(m, np.where(np.isfinite(e), _near_int(e), np.inf))
    fragile = front & ~reach & (m < FRAGILE)
    fragile |= np.abs(Z - znear) / np.maximum(1.0, np.abs(Z)) < FRAGILE
    return vis, fragile


def visibility_count(points, cams, rho, filter_px):
    """Visible frequency of each point over the views (counts [m] int64) and the number of views in
    which its decision is fragile."""
    m = np.asarray(points).shape[1]
    cnt = np.zeros(m, np.int64)
    frag = np.zeros(m, np.int64)
    for cam in cams:
        v, f = visible(points, cam, rho, filter_px)
        cnt += v
        frag += f
    return cnt, frag


def crop_volume(points, counts, tau_min, T):
    """Points seen in at least tau_min views: (keep [m] bool, ground xy [2][k] of the kept points in id
    order, h_min, h_max) with (x, y, h) = T p (NaN heights when none is kept)."""
    P = np.asarray(points, np.float32).astype(np.float64)
    T = np.asarray(T, np.float64).reshape(3, 4)
    keep = np.asarray(counts) >= tau_min
    G = T[:, :3] @ P[:, keep] + T[:, 3:4]
    if keep.any():
        return keep, G[:2], float(G[2].min()), float(G[2].max())
    return keep, G[:2], float("nan"), float("nan")
