"""FP64 CPU reference of the 2DGS surfel rasterizer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2411_00771_amd``) and never imports it; the two meet only in the
seeded input generators.  Each wrapper names the paper passage it follows; the
arithmetic lives in ``cgv2_oracle.cpp`` (projection, binning, Eq. 1 blending,
its reverse mode, SSIM, the Eq. 3 contribution) and in :func:`densify_stats`,
:func:`average_contribution` and :func:`trim_threshold` below (Eq. 2, the
elongation rate of Sec. 3.2, Eq. 4 and the trimming bound of Sec. 3.3) and in
:func:`densify_actions` / :func:`densify_apply` (the densification action).
``oracle.visibility`` holds the visibility-frequency crop-volume estimate of Sec. 4.

Parity-unpinned readings (the paper fixes none of them; they are pinned to the
mathematics instead): pixel-centre sampling, the screen low-pass filter width,
the lossless opacity-aware cutoff, the intersection depth of the 3D branch, the
median-depth rule, the SH offset/clamp, the per-view DGD averages, the
elongation threshold, the 2DGS view-space gradient, the contribution region
(the pixels where a surfel is blended) and the percentile bound of the trim.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cgv2_oracle.cpp")
_LIB = os.path.join(_HERE, "libcgv2_oracle.so")
_lib = None

F_VISIBLE, F_NEAR, F_OPACITY, F_BEHIND, F_NONFINITE, F_LOWPASS = 1, 2, 4, 8, 16, 32
F_CULLED = F_NEAR | F_OPACITY | F_BEHIND | F_NONFINITE

LAMBDA_SSIM = 0.2


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _scene64(scene):
    return dict(mean=_d(scene.mean), log_scale=_d(scene.log_scale), quat=_d(scene.quat),
                opacity_logit=_d(scene.opacity_logit), sh=_d(scene.sh), sh_degree=scene.sh_degree)


def _params(scene):
    """Accepts a Scene or a dict of float64 arrays (used by the finite-difference tests)."""
    if isinstance(scene, dict):
        return {k: (_d(v) if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    return _scene64(scene)


# ---------------------------------------------------------------------------------------------
# Projection (2DGS surfels, Sec. 3.1; low-pass filter, Sec. 3.2)
# ---------------------------------------------------------------------------------------------

def project(scene, cam):
    P = _params(scene)
    n = P["mean"].shape[1]
    out = dict(M=np.zeros((n, 9)), rgb=np.zeros((n, 3)), rgb_raw=np.zeros((n, 3)), normal=np.zeros((n, 3)),
               opacity=np.zeros(n), k2=np.zeros(n), bbox=np.zeros((n, 4)), pix_rect=np.zeros((n, 4), np.int32),
               tile_rect=np.zeros((n, 4), np.int32), radius=np.zeros(n), flags=np.zeros(n, np.int32))
    c = _d(cam.as_array())
    rc = lib().orc_project(ctypes.c_int64(n), ctypes.c_int(P["sh_degree"]), _p(P["mean"]), _p(P["log_scale"]),
                           _p(P["quat"]), _p(P["opacity_logit"]), _p(P["sh"]), _p(c),
                           *[_p(out[k]) for k in ("M", "rgb", "rgb_raw", "normal", "opacity", "k2", "bbox",
                                                  "pix_rect", "tile_rect", "radius", "flags")])
    assert rc == 0
    out["depth"] = out["M"][:, 8].copy()
    out["depth32"] = out["depth"].astype(np.float32)
    return out


def bin_tiles(tile_rect, depth32, width, height, keep=None):
    """Per-tile lists ordered by (float32 depth bits, id): every tile of each surfel's tile rect, or,
    with ``keep`` (one byte per rect tile in the order of :func:`rect_tiles`), those it marks."""
    tile_rect = np.ascontiguousarray(tile_rect, np.int32)
    depth32 = np.ascontiguousarray(depth32, np.float32)
    keep = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    n = tile_rect.shape[0]
    ntiles = ((width + 15) // 16) * ((height + 15) // 16)
    offsets = np.zeros(ntiles + 1, np.int64)
    L = lib()
    L.orc_bin.restype = ctypes.c_int64
    K = L.orc_bin(ctypes.c_int64(n), width, height, _p(tile_rect), _p(depth32), _p(keep), _p(offsets), None,
                  ctypes.c_int64(0))
    ids = np.zeros(max(K, 1), np.int32)
    L.orc_bin(ctypes.c_int64(n), width, height, _p(tile_rect), _p(depth32), _p(keep), _p(offsets), _p(ids),
              ctypes.c_int64(K))
    return offsets, ids[:K]


def rect_tiles(tile_rect, width):
    """(surfel, tile) of every tile of every surfel's tile rect, in (surfel, row, column) order."""
    r = np.asarray(tile_rect, np.int64)
    w = np.maximum(r[:, 2] - r[:, 0], 0)
    h = np.maximum(r[:, 3] - r[:, 1], 0)
    cnt = w * h
    sid = np.repeat(np.arange(r.shape[0]), cnt)
    k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tx = r[sid, 0] + k % np.maximum(w[sid], 1)
    ty = r[sid, 1] + k // np.maximum(w[sid], 1)
    return sid, ty * ((width + 15) // 16) + tx


def tile_reach(proj):
    """The list rule: which tiles of each surfel's tile rect its cutoff region rho <= k2 can reach
    (evaluated with k2 enlarged by 2e-3 relative + 2e-3 and the tile's pixel-sample box padded by
    1/64 px), and which of these decisions are fragile (flip when the enlarged cutoff moves by 1e-5
    relative and the pad by 1e-3 px).  Arrays over the rect tiles in :func:`rect_tiles` order."""
    tr = np.ascontiguousarray(proj["tile_rect"], np.int32)
    n = tr.shape[0]
    L = lib()
    L.orc_tile_reach.restype = ctypes.c_int64
    M, k2 = _d(proj["M"]), _d(proj["k2"])
    total = L.orc_tile_reach(ctypes.c_int64(n), _p(M), _p(k2), _p(tr), None, None)
    keep = np.zeros(max(total, 1), np.uint8)
    fragile = np.zeros(max(total, 1), np.uint8)
    L.orc_tile_reach(ctypes.c_int64(n), _p(M), _p(k2), _p(tr), _p(keep), _p(fragile))
    return keep[:total].astype(bool), fragile[:total].astype(bool)


def bin_view(proj, cam):
    """Per-tile lists of one view under the list rule of :func:`tile_reach`.  Returns (offsets, ids,
    info) with info = dict(rect_total: entries of the plain tile-rect lists, fragile: int64 keys
    tile * n + surfel of the fragile (tile, surfel) decisions)."""
    keep, fragile = tile_reach(proj)
    offsets, ids = bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height, keep=keep)
    sid, tile = rect_tiles(proj["tile_rect"], cam.width)
    n = proj["tile_rect"].shape[0]
    return offsets, ids, dict(rect_total=int(keep.size), fragile=tile[fragile] * n + sid[fragile])


# ---------------------------------------------------------------------------------------------
# Eq. 1 front-to-back blending
# ---------------------------------------------------------------------------------------------

def _img_buffers(cam):
    H, W = cam.height, cam.width
    return dict(rgb=np.zeros((3, H, W)), depth=np.zeros((H, W)), depth_med=np.zeros((H, W)),
                normal=np.zeros((3, H, W)), alpha=np.zeros((H, W)), T=np.zeros((H, W)))


def render(proj, cam, offsets, ids):
    out = _img_buffers(cam)
    H, W = cam.height, cam.width
    out.update(last=np.zeros((H, W), np.int64), med=np.zeros((H, W), np.int64), margin=np.zeros((H, W)),
               sig=np.zeros((H, W), np.uint64))
    counters = np.zeros(2, np.int64)
    n = proj["M"].shape[0]
    rc = lib().orc_render(ctypes.c_int64(n), _p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]), _p(proj["opacity"]),
                          _p(_d(cam.as_array())), _p(np.ascontiguousarray(offsets, np.int64)),
                          _p(np.ascontiguousarray(ids, np.int32)), _p(out["rgb"]), _p(out["depth"]),
                          _p(out["depth_med"]), _p(out["normal"]), _p(out["alpha"]), _p(out["T"]), _p(out["last"]),
                          _p(out["med"]), _p(counters), _p(out["margin"]), _p(out["sig"]))
    assert rc == 0
    out["n_eval"], out["n_con"] = int(counters[0]), int(counters[1])
    return out


def render_tiles(proj, cam, offsets, ids, tiles):
    """Render only the listed tiles: returns [ntiles, 16, 16, 13] (rgb, D, Dmed, N, A, T, margin, id of the
    median fragment, id of the last contributor; -1 where none)."""
    tiles = np.ascontiguousarray(tiles, np.int32)
    out = np.full((len(tiles), 16, 16, 13), np.nan)
    counters = np.zeros(2, np.int64)
    lib().orc_render_tiles(_p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]), _p(proj["opacity"]),
                           _p(_d(cam.as_array())), _p(np.ascontiguousarray(offsets, np.int64)),
                           _p(np.ascontiguousarray(ids, np.int32)), ctypes.c_int64(len(tiles)), _p(tiles),
                           _p(out), _p(counters))
    return out, int(counters[0]), int(counters[1])


def render_brute(proj, cam):
    out = _img_buffers(cam)
    out["med_id"] = np.zeros((cam.height, cam.width), np.int64)
    n = proj["M"].shape[0]
    lib().orc_render_brute(ctypes.c_int64(n), _p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]),
                           _p(proj["opacity"]), _p(proj["flags"]), _p(_d(cam.as_array())), _p(out["rgb"]),
                           _p(out["depth"]), _p(out["depth_med"]), _p(out["normal"]), _p(out["alpha"]), _p(out["T"]),
                           _p(out["med_id"]))
    return out


def render_bwd(proj, cam, offsets, ids, d_rgb=None, d_depth=None, d_depth_med=None, d_normal=None, d_alpha=None,
               tile_mask=None):
    n = proj["M"].shape[0]
    g = dict(M=np.zeros((n, 9)), rgb=np.zeros((n, 3)), normal=np.zeros((n, 3)), opacity=np.zeros(n))
    counters = np.zeros(1, np.int64)
    up = [None if a is None else _d(a) for a in (d_rgb, d_depth, d_depth_med, d_normal, d_alpha)]
    lib().orc_render_bwd(ctypes.c_int64(n), _p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]), _p(proj["opacity"]),
                         _p(_d(cam.as_array())), _p(np.ascontiguousarray(offsets, np.int64)),
                         _p(np.ascontiguousarray(ids, np.int32)), *[_p(a) for a in up], _p(g["M"]), _p(g["rgb"]),
                         _p(g["normal"]), _p(g["opacity"]), _p(counters),
                         None if tile_mask is None else _p(np.ascontiguousarray(tile_mask, np.uint8)))
    g["n_pairs"] = int(counters[0])
    return g


def contribution(proj, cam, offsets, ids, gamma=0.5, fragile=-1.0):
    """Per-surfel contribution in one view, Sec. 3.3 Eq. 3: C = (1/|P|) sum_P alpha^gamma T^(1-gamma) over
    the pixels P where the surfel is blended (T = transmittance in front of it); C = 0 when P is empty.
    'fragile' counts, per surfel, the pixels where it is evaluated and whose decision margin is below the
    given bound (each can move its count by at most 1 and its sum by at most one term); 'err' bounds, to
    first order, the error an FP32 evaluation of the terms makes in 'sum' (FP32 error model of alpha and
    of the accumulated T, as behind the decision margins)."""
    n = proj["M"].shape[0]
    out = dict(sum=np.zeros(n), cnt=np.zeros(n, np.int64), fragile=np.zeros(n, np.int32), err=np.zeros(n))
    lib().orc_contribution(ctypes.c_int64(n), _p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]),
                           _p(proj["opacity"]), _p(_d(cam.as_array())), _p(np.ascontiguousarray(offsets, np.int64)),
                           _p(np.ascontiguousarray(ids, np.int32)), ctypes.c_double(gamma), ctypes.c_double(fragile),
                           _p(out["sum"]), _p(out["cnt"]), _p(out["fragile"]), _p(out["err"]))
    out["C"] = np.where(out["cnt"] > 0, out["sum"] / np.maximum(out["cnt"], 1), 0.0)
    return out


def contribution_brute(proj, cam, gamma=0.5):
    """Eq. 3 with every surviving surfel blended at every pixel (no tiles)."""
    n = proj["M"].shape[0]
    out = dict(sum=np.zeros(n), cnt=np.zeros(n, np.int64))
    lib().orc_contribution_brute(ctypes.c_int64(n), _p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]),
                                 _p(proj["opacity"]), _p(np.ascontiguousarray(proj["flags"], np.int32)),
                                 _p(_d(cam.as_array())), ctypes.c_double(gamma), _p(out["sum"]), _p(out["cnt"]))
    out["C"] = np.where(out["cnt"] > 0, out["sum"] / np.maximum(out["cnt"], 1), 0.0)
    return out


def average_contribution(per_view):
    """Eq. 4: the mean of the single-view contributions over the views of the block."""
    return np.mean(np.stack([np.asarray(c, np.float64) for c in per_view]), axis=0)


def trim_threshold(C, ratio):
    """Sec. 3.3 trimming: the bound is the floor(ratio (n - 1))-th smallest contribution (0-based; the
    'lower' percentile); every surfel at or below it is removed.  Returns (bound, mask)."""
    C = np.asarray(C)
    k = int(np.floor(ratio * (C.size - 1)))
    bound = np.sort(C, kind="stable")[k]
    return bound, C <= bound


def _rotation(q):
    """Rotation matrices [n][3][3] of (unnormalised) quaternions q[4][n] = (w, x, y, z)."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q, axis=0)
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def densify_actions(cand, remove, log_scale, opacity_logit, dense_scale, min_opacity):
    """Per-surfel action: 3 remove (trimmed, Sec. 3.3, or opacity below min_opacity), else for the
    densification candidates of Sec. 3.2 (DGD high-gradient and not elongated) 1 clone when
    max(s_u, s_v) <= dense_scale and 2 split otherwise, else 0 keep."""
    s_max = np.exp(np.asarray(log_scale, np.float64)).max(axis=0)
    o = 1 / (1 + np.exp(-np.asarray(opacity_logit, np.float64)))
    act = np.where(np.asarray(cand, bool), np.where(s_max <= dense_scale, 1, 2), 0)
    rm = np.asarray(remove, bool) if remove is not None else np.zeros(act.shape, bool)
    return np.where(rm | (o < min_opacity), 3, act).astype(np.int32)


def densify_apply(P, actions, z, shrink=1.6):
    """The new surfel set: survivors (keep, clone) in id order, then for every clone (a copy) or split
    (two children) in id order its new surfels.  Child c of a split surfel sits at
    mu + R (s_u z[i, c, 0], s_v z[i, c, 1], 0) in its own plane and has its scales divided by 'shrink';
    rotation, opacity and SH are copied.  P uses the generators' planar layout (sh [K][3][n])."""
    act = np.asarray(actions)
    R = _rotation(P["quat"])
    s = np.exp(np.asarray(P["log_scale"], np.float64))
    surv = np.flatnonzero((act == 0) | (act == 1))
    out = {k: [] for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}

    def take(idx, mean=None, log_scale=None):
        out["mean"].append(np.asarray(P["mean"], np.float64)[:, idx] if mean is None else mean)
        out["log_scale"].append(np.asarray(P["log_scale"], np.float64)[:, idx] if log_scale is None else log_scale)
        out["quat"].append(np.asarray(P["quat"], np.float64)[:, idx])
        out["opacity_logit"].append(np.asarray(P["opacity_logit"], np.float64)[idx])
        out["sh"].append(np.asarray(P["sh"], np.float64)[:, :, idx])

    take(surv)
    for i in np.flatnonzero((act == 1) | (act == 2)):
        if act[i] == 1:
            take(np.array([i]))
            continue
        for c in range(2):
            local = np.array([s[0, i] * z[i, c, 0], s[1, i] * z[i, c, 1], 0.0])
            mu = np.asarray(P["mean"], np.float64)[:, i] + R[i] @ local
            take(np.array([i]), mean=mu[:, None],
                 log_scale=(np.asarray(P["log_scale"], np.float64)[:, i] - np.log(shrink))[:, None])
    res = {k: np.concatenate(v, axis=-1) for k, v in out.items()}
    res["sh_degree"] = P["sh_degree"]
    return res


def densify_slots(actions):
    """Output slots of a plan, by the order :func:`densify_apply` defines: dst[0][i] the slot of surfel i
    itself (keep, clone), dst[1][i] the first slot of its new surfel(s), -1 where none; and per output
    slot its source id and kind (0 survivor, 1 clone copy, 2 / 3 split child 0 / 1)."""
    act = np.asarray(actions)
    n = act.shape[0]
    dst = np.full((2, n), -1, np.int64)
    src, kind = [], []
    for i in range(n):
        if act[i] in (0, 1):
            dst[0, i] = len(src)
            src.append(i)
            kind.append(0)
    for i in range(n):
        if act[i] == 1:
            dst[1, i] = len(src)
            src.append(i)
            kind.append(1)
        elif act[i] == 2:
            dst[1, i] = len(src)
            src += [i, i]
            kind += [2, 3]
    return dst, np.array(src, np.int64), np.array(kind, np.int64)


def project_bwd(scene, cam, g):
    P = _params(scene)
    out = dict(mean=np.zeros_like(P["mean"]), log_scale=np.zeros_like(P["log_scale"]), quat=np.zeros_like(P["quat"]),
               opacity_logit=np.zeros_like(P["opacity_logit"]), sh=np.zeros_like(P["sh"]))
    n = P["mean"].shape[1]
    lib().orc_project_bwd(ctypes.c_int64(n), ctypes.c_int(P["sh_degree"]), _p(P["mean"]), _p(P["log_scale"]),
                          _p(P["quat"]), _p(P["opacity_logit"]), _p(P["sh"]), _p(_d(cam.as_array())), _p(_d(g["M"])),
                          _p(_d(g["rgb"])), _p(_d(g["normal"])), _p(_d(g["opacity"])), _p(out["mean"]),
                          _p(out["log_scale"]), _p(out["quat"]), _p(out["opacity_logit"]), _p(out["sh"]))
    return out


def viewspace_grad(M, dM, width, height, ndc=True):
    """Gradient w.r.t. a rigid screen translation of the splat's image (the 2DGS analogue of the
    view-space position gradient of Sec. 3.1): row1 += dx * row3, row2 += dy * row3 of M."""
    M = np.asarray(M).reshape(-1, 3, 3)
    dM = np.asarray(dM).reshape(-1, 3, 3)
    g = np.stack([(dM[:, 0, :] * M[:, 2, :]).sum(1), (dM[:, 1, :] * M[:, 2, :]).sum(1)], 1)
    if ndc:
        g = g * np.array([width / 2.0, height / 2.0])
    return g


def eval_pairs(M, opacity, xy):
    """Ray-splat evaluation of m (surfel, sample) pairs (Sec. 3.1, Eq. 1's alpha) with the first-order
    FP32 error bounds the decision margins use.  M [m][9], opacity [m], xy [m][2] -> dict of rho3, rho2,
    alpha, drho3, drho2, dalpha_rel (relative), is3d, clamped."""
    M, o, xy = _d(M).reshape(-1, 9), _d(opacity).ravel(), _d(xy).reshape(-1, 2)
    m = M.shape[0]
    out = np.zeros((m, 8))
    lib().orc_eval_pairs(ctypes.c_int64(m), _p(M), _p(o), _p(xy), _p(out))
    keys = ("rho3", "rho2", "alpha", "drho3", "drho2", "dalpha_rel")
    res = {k: out[:, i] for i, k in enumerate(keys)}
    res["is3d"], res["clamped"] = out[:, 6] > 0, out[:, 7] > 0
    return res


def blend_trace(proj, cam, ids, x, y, cap=4096):
    """The contributing fragments of the pixel sample (x, y) over the list ids, in blend order (Eq. 1):
    (frag [k][5] = id, alpha, T in front, relative bound of alpha, relative bound of T behind, margin)."""
    ids = np.ascontiguousarray(ids, np.int32)
    frag = np.zeros((cap, 5))
    margin = np.zeros(1)
    L = lib()
    L.orc_blend_trace.restype = ctypes.c_int64
    k = L.orc_blend_trace(_p(proj["M"]), _p(proj["rgb"]), _p(proj["normal"]), _p(proj["opacity"]),
                          _p(_d(cam.as_array())), _p(ids), ctypes.c_int64(len(ids)), ctypes.c_double(x),
                          ctypes.c_double(y), _p(frag), ctypes.c_int64(cap), _p(margin))
    return frag[:min(k, cap)], float(margin[0])


def set_threads(t: int) -> int:
    """Threads of the oracle's OpenMP loops (t <= 0 leaves them); returns the number in effect."""
    return int(lib().orc_set_threads(int(t)))


def sh_eval(deg, dirs):
    dirs = _d(dirs)
    m = dirs.shape[0]
    K = (deg + 1) ** 2
    Y = np.zeros((m, K))
    dY = np.zeros((m, K, 3))
    lib().orc_sh_eval(ctypes.c_int(deg), ctypes.c_int64(m), _p(dirs), _p(Y), _p(dY))
    return Y, dY


def ssim_loss(img, target, lam=LAMBDA_SSIM):
    """(1 - lam) L1 + lam (1 - SSIM) (Sec. 3.1), its total gradient, its SSIM-only gradient and the
    per-pixel SSIM map."""
    img, target = _d(img), _d(target)
    _, H, W = img.shape
    parts = np.zeros(3)
    dt, ds, mp = np.zeros_like(img), np.zeros_like(img), np.zeros_like(img)
    lib().orc_ssim_loss(H, W, _p(img), _p(target), ctypes.c_double(lam), _p(parts), _p(dt), _p(ds), _p(mp))
    return dict(loss=parts[0], l1=parts[1], ssim=parts[2], d_total=dt, d_ssim=ds, map=mp)


# ---------------------------------------------------------------------------------------------
# Decomposed-gradient densification statistics (Eq. 2) and the elongation filter (Sec. 3.2)
# ---------------------------------------------------------------------------------------------

def densify_stats(g_tot, g_ssim, visible, radius, log_scale, state, omega=0.9, eta_min=0.05, grad_threshold=2e-4,
                  lowpass=None):
    """One view's update of the densification state.

    g_tot, g_ssim: (n, 2) view-space gradients of the total loss and of the SSIM term.
    Eq. 2: scale = max(omega * |g_tot|_avg / |g_ssim|_avg, 1) with both averages taken over the
    surfels visible in this view; the densification gradient is scale * |g_ssim|.
    Elongation rate eta = min(s_u, s_v) / max(s_u, s_v); eta < eta_min excludes a surfel from
    clone/split.  State: accum_dgd, accum_total, max_radius, denom (float64 / int64 arrays).
    """
    vis = np.asarray(visible, bool)
    nt = np.sqrt((np.asarray(g_tot, np.float64) ** 2).sum(1))
    ns = np.sqrt((np.asarray(g_ssim, np.float64) ** 2).sum(1))
    a_tot = nt[vis].sum()
    a_ssim = ns[vis].sum()
    scale = max(omega * a_tot / a_ssim, 1.0) if a_ssim > 0 else 1.0
    state["accum_dgd"] = state["accum_dgd"] + np.where(vis, scale * ns, 0.0)
    state["accum_total"] = state["accum_total"] + np.where(vis, nt, 0.0)
    state["denom"] = state["denom"] + vis.astype(np.int64)
    state["max_radius"] = np.where(vis, np.maximum(state["max_radius"], radius), state["max_radius"])
    s = np.exp(np.asarray(log_scale, np.float64))
    eta = s.min(0) / s.max(0)
    avg = np.where(state["denom"] > 0, state["accum_dgd"] / np.maximum(state["denom"], 1), 0.0)
    high = avg >= grad_threshold
    elong = eta < eta_min
    lp = np.zeros_like(vis) if lowpass is None else np.asarray(lowpass, bool)
    cand = high & ~elong
    counters = np.array([vis.sum(), high.sum(), elong.sum(), (high & elong).sum(), (vis & lp).sum(), cand.sum(),
                         0, 0], np.int64)
    mask = (high * 1) | (elong * 2) | (cand * 4) | ((vis & lp) * 8)
    return dict(scale=scale, a_tot=a_tot, a_ssim=a_ssim, eta=eta, mask=mask.astype(np.uint8), counters=counters)


def new_densify_state(n):
    return dict(accum_dgd=np.zeros(n), accum_total=np.zeros(n), max_radius=np.zeros(n), denom=np.zeros(n, np.int64))


# ---------------------------------------------------------------------------------------------
# Whole-view compositions used by tests
# ---------------------------------------------------------------------------------------------

def forward_view(scene, cam):
    proj = project(scene, cam)
    offsets, ids, _ = bin_view(proj, cam)
    img = render(proj, cam, offsets, ids)
    return proj, offsets, ids, img


def backward_view(scene, cam, proj, offsets, ids, upstream, ndc=True):
    """Parameter gradients, plus the view-space gradients of the total upstream and of the
    SSIM-only colour upstream ``d_rgb_ssim`` (the two sources of Eq. 2)."""
    up = {k: v for k, v in upstream.items() if k != "d_rgb_ssim"}
    g = render_bwd(proj, cam, offsets, ids, **up)
    pg = project_bwd(scene, cam, g)
    out = dict(params=pg, record=g, g_total=viewspace_grad(proj["M"], g["M"], cam.width, cam.height, ndc))
    if upstream.get("d_rgb_ssim") is not None:
        gs = render_bwd(proj, cam, offsets, ids, d_rgb=upstream["d_rgb_ssim"])
        out["g_ssim"] = viewspace_grad(proj["M"], gs["M"], cam.width, cam.height, ndc)
    return out
