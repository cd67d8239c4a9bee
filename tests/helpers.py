"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and fetch numpy
arrays, and compare against the FP64 oracle with the decision-margin policy."""
from __future__ import annotations

import numpy as np

FRAGILE = 1e-5          # pixels whose smallest relative decision margin is below this are excluded
IMG_TOL = 1e-4          # max abs error on rgb / alpha / normal / T
GRAD_REL = 1e-3         # per-group ||d - ref|| / ||ref||


def gpu_forward(scene, cams, capacity=None, target=None):
    import torch
    from paper_2411_00771_amd import raster
    params = raster.Params.from_scene(scene)
    eng = raster.Engine(scene.n, cams[0].width, cams[0].height, len(cams), capacity=capacity)
    cs = eng.cams(cams)
    eng.status.zero_()
    eng.forward(params, cs)
    torch.cuda.synchronize()
    return eng, params, cs


def fetch_proj(eng):
    V, n = eng.V, eng.n
    rec = eng.rec.view(V, n, 24).cpu().numpy()
    rect = eng.rect.view(V, n, 4).cpu().numpy().view(np.uint16).astype(np.int32)
    return dict(rec=rec, rect=rect, radius=eng.radius.view(V, n).cpu().numpy(),
                flags=eng.flags.view(V, n).cpu().numpy().astype(np.int32))


def fetch_bins(eng):
    ranges = eng.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    K = int(ranges[-1])
    ids = eng.ids[:K].cpu().numpy().view(np.uint32).astype(np.int64)
    return ranges, ids


def fetch_img(eng, v=0):
    g = lambda t: t[v].cpu().numpy()
    return dict(rgb=g(eng.rgb), depth=g(eng.depth), depth_med=g(eng.depth_med), normal=g(eng.normal),
                alpha=g(eng.alpha), T=g(eng.T_final), last=g(eng.last).view(np.uint32).astype(np.int64),
                med=g(eng.med).view(np.uint32).astype(np.int64))


def depth_scale(img):
    return max(1.0, float(np.abs(img["depth"]).max()))


def compare_images(gpu, ref, margin, tol=IMG_TOL, fragile=FRAGILE, max_fragile_frac=1e-3):
    """Max abs errors on the non-fragile pixels; asserts the tolerance and the fragile fraction."""
    ok = margin >= fragile
    frac = 1.0 - ok.mean()
    assert frac <= max_fragile_frac, f"fragile pixel fraction {frac:.2e}"
    errs = {}
    zs = max(1.0, float(np.abs(ref["depth_med"]).max()))
    for k in ("rgb", "normal"):
        errs[k] = float(np.abs(gpu[k] - ref[k])[:, ok].max()) if ok.any() else 0.0
    for k in ("alpha", "T"):
        errs[k] = float(np.abs(gpu[k] - ref[k])[ok].max()) if ok.any() else 0.0
    for k in ("depth", "depth_med"):
        errs[k] = float(np.abs(gpu[k] - ref[k])[ok].max()) / zs if ok.any() else 0.0
    for k, e in errs.items():
        assert e <= tol, f"{k}: max err {e:.3e} > {tol}"
    return errs, frac


def grad_close(name, g, ref, rel=GRAD_REL):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(ref)
    err = np.linalg.norm(g - ref) / max(nr, 1e-30)
    assert err <= rel, f"{name}: relative error {err:.3e} > {rel} (|ref| {nr:.3e})"
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    bad = np.abs(g - ref) > rel * (np.abs(ref) + 0.01 * rms) + 1e-30
    # elementwise: allow a handful of outliers from fp32 cancellation, never more than 0.1 %
    assert bad.mean() <= 1e-3, f"{name}: {bad.sum()} elements outside the elementwise bound"
    return err


def compare_lists(ranges, ids, po, cam, P=None, v=0, max_excluded=None):
    """GPU tile lists against the oracle's (its own projection `po`, the reach rule of
    ``oracle.bin_view``), entry for entry and in order.  Left out on both sides: the surfels whose
    projection decisions differ (visibility, tile rect or depth key; only when the GPU projection `P` is
    given) and the (tile, surfel) pairs whose reach decision the oracle marks fragile.  Returns the
    counts left out."""
    import oracle
    off, oids, info = oracle.bin_view(po, cam)
    n = po["tile_rect"].shape[0]
    T = len(off) - 1
    assert len(ranges) == T + 1
    excl = np.zeros(n, bool)
    if P is not None:
        vis_g, vis_o = (P["flags"][v] & 1) > 0, (po["flags"] & 1) > 0
        excl |= vis_g != vis_o
        both = vis_g & vis_o
        excl |= both & (P["rect"][v] != po["tile_rect"]).any(1)
        kg = P["rec"][v, :, 11].astype(np.float32).view(np.uint32)
        excl |= both & (kg != po["depth32"].view(np.uint32))
    fr = np.sort(np.asarray(info["fragile"], np.int64))

    def left_out(rng, lst):
        tile = np.repeat(np.arange(T, dtype=np.int64), np.diff(rng))
        key = tile * n + lst
        pos = np.searchsorted(fr, key)
        hit = (pos < fr.size) & (fr[np.minimum(pos, max(fr.size - 1, 0))] == key) if fr.size else np.zeros(key.size, bool)
        return excl[lst] | hit, tile

    mg, tg = left_out(np.asarray(ranges, np.int64), np.asarray(ids, np.int64))
    mo, to = left_out(off, np.asarray(oids, np.int64))
    assert np.array_equal(np.bincount(tg[~mg], minlength=T), np.bincount(to[~mo], minlength=T)), "per-tile counts"
    assert np.array_equal(np.asarray(ids)[~mg], np.asarray(oids)[~mo]), "list order"
    out = dict(surfels=int(excl.sum()), fragile_pairs=int(fr.size), entries_g=int(mg.sum()), entries_o=int(mo.sum()),
               rect_total=info["rect_total"], listed=int(len(oids)))
    if max_excluded is not None:
        assert out["surfels"] + out["fragile_pairs"] <= max_excluded, out
    return out


def compare_sampled_tiles(eng, ref, tiles, v=0, tol=IMG_TOL, fragile=FRAGILE):
    """Every output of view v on the tiles the oracle rendered one by one (``oracle.render_tiles``):
    rgb, expected and median depth (relative to the tiles' depth scale), normal, alpha, T, and the ids of
    the median fragment and the last contributor, on the pixels whose decisions are not fragile.
    Returns (worst error per output, fragile pixels, pixels)."""
    W, H, tx = eng.W, eng.H, eng.tiles_x
    img = fetch_img(eng, v)
    ranges, ids = fetch_bins(eng)
    ranges = ranges[v * eng.tiles:(v + 1) * eng.tiles + 1]
    ids_ext = np.append(ids, -1)
    worst = dict(rgb=0.0, depth=0.0, depth_med=0.0, normal=0.0, alpha=0.0, T=0.0, med=0, last=0)
    zs = max(1.0, float(np.nanmax(np.abs(ref[..., 4]))))
    nfr, total = 0, 0
    for s, t in enumerate(tiles):
        oy, ox = (t // tx) * 16, (t % tx) * 16
        h, w = min(16, H - oy), min(16, W - ox)
        r = ref[s, :h, :w]
        ok = r[..., 10] >= fragile
        nfr += int((~ok).sum())
        total += h * w
        win = (slice(oy, oy + h), slice(ox, ox + w))
        diff = lambda g, k: float(np.abs(g - r[..., k])[ok].max(initial=0))
        worst["rgb"] = max(worst["rgb"], *(diff(img["rgb"][c][win], c) for c in range(3)))
        worst["normal"] = max(worst["normal"], *(diff(img["normal"][c][win], 5 + c) for c in range(3)))
        worst["depth"] = max(worst["depth"], diff(img["depth"][win], 3) / zs)
        worst["depth_med"] = max(worst["depth_med"], diff(img["depth_med"][win], 4) / zs)
        worst["alpha"] = max(worst["alpha"], diff(img["alpha"][win], 8))
        worst["T"] = max(worst["T"], diff(img["T"][win], 9))
        start = ranges[t]
        med = img["med"][win]
        med_id = np.where(med == 0xffffffff, -1, ids_ext[np.minimum(med, len(ids))])
        last = img["last"][win]
        last_id = np.where(last > start, ids_ext[np.minimum(np.maximum(last - 1, 0), len(ids))], -1)
        worst["med"] += int((med_id != r[..., 11])[ok].sum())
        worst["last"] += int((last_id != r[..., 12])[ok].sum())
    for k in ("rgb", "depth", "depth_med", "normal", "alpha", "T"):
        assert worst[k] <= tol, f"{k}: max err {worst[k]:.3e} > {tol}"
    assert worst["med"] == 0 and worst["last"] == 0, worst
    return worst, nfr, total
