"""HIP path vs the FP64 oracle on the tiny workload (4,096 surfels, 128x128) and edge cases.

Every call goes through the C ABI (libcgv2r.so).  Tolerances: images 1e-4 max abs on pixels whose
decision margins are not fragile; per-tile lists bit-exact; gradients 1e-3 relative per group.
"""
import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes
from tests.helpers import (FRAGILE, compare_images, compare_lists, fetch_bins, fetch_img, fetch_proj, gpu_forward,
                           grad_close)

pytestmark = pytest.mark.gpu


def _oracle_all(sc, cam):
    return oracle.forward_view(sc, cam)


@pytest.fixture(scope="module")
def tiny(cuda):
    w = scenes.workload(0)
    sc, cam, tgt = w["scene"], w["cameras"][0], w["targets"][0]
    eng, params, cs = gpu_forward(sc, [cam], capacity=1 << 16)
    po, off, ids, io = _oracle_all(sc, cam)
    return dict(sc=sc, cam=cam, tgt=tgt, eng=eng, params=params, cs=cs, po=po, off=off, ids=ids, io=io)


def test_project_matches_oracle(tiny):
    P = fetch_proj(tiny["eng"])
    po = tiny["po"]
    rec, fl = P["rec"][0], P["flags"][0]
    cull = 2 | 4 | 8 | 16
    assert np.array_equal(fl & cull, po["flags"] & cull)
    vis_o = (po["flags"] & 1) > 0
    vis = (fl & 1) > 0
    assert np.array_equal(vis, vis_o)
    v = vis
    assert np.abs(rec[v, 13:16] - po["rgb"][v]).max() <= 2e-6
    assert np.abs(rec[v, 16:19] - po["normal"][v]).max() <= 1e-6
    assert np.abs(rec[v, 12] - po["opacity"][v]).max() <= 1e-6
    assert np.array_equal(rec[v, 11].astype(np.float32).view(np.uint32), po["depth32"][v].view(np.uint32))
    M = po["M"][v]
    cx = rec[v, 0].astype(np.float64) + rec[v, 2]
    cy = rec[v, 1].astype(np.float64) + rec[v, 3]
    assert np.abs(cx - M[:, 2] / M[:, 8]).max() <= 1e-5
    assert np.abs(cy - M[:, 5] / M[:, 8]).max() <= 1e-5
    assert np.array_equal(P["rect"][0][v], po["tile_rect"][v])
    assert np.abs(P["radius"][0][v] / po["radius"][v] - 1).max() <= 1e-5
    # inverse homography: rho_3d and the intersection depth at offsets from the centre
    rng = np.random.default_rng(0)
    for _ in range(4):
        d = rng.normal(size=2) * 2.0
        xr, yr = d
        a11, a12, a21, a22, w0, w1, w2 = [rec[v, k].astype(np.float64) for k in range(4, 11)]
        P1, P2, w = a11 * xr + a12 * yr, a21 * xr + a22 * yr, w0 + w1 * xr + w2 * yr
        rho = (P1 ** 2 + P2 ** 2) / w ** 2
        zf = rec[v, 11] * w0 / w
        x, y = M[:, 2] / M[:, 8] + xr, M[:, 5] / M[:, 8] + yr
        a = x[:, None] * M[:, 6:9] - M[:, 0:3]
        b = y[:, None] * M[:, 6:9] - M[:, 3:6]
        p = np.cross(a, b)
        u, vv = p[:, 0] / p[:, 2], p[:, 1] / p[:, 2]
        assert np.abs(rho / (u * u + vv * vv) - 1).max() <= 1e-4
        zref = M[:, 6] * u + M[:, 7] * vv + M[:, 8]
        assert np.abs(zf / zref - 1).max() <= 1e-5
    # low-pass flag: equal wherever the two branches are not within rounding at that sample
    assert np.mean((fl & 32) != (po["flags"] & 32)) <= 1e-3


def test_bin_sort_bit_exact(tiny):
    eng = tiny["eng"]
    P = fetch_proj(eng)
    ranges, ids = fetch_bins(eng)
    # the oracle's own projection and lists (reach rule); its rects and keys equal the GPU's here
    r = compare_lists(ranges, ids, tiny["po"], tiny["cam"], P=P, max_excluded=2)
    assert r["surfels"] == 0
    # the staging holds every tile of every rect; the lists keep the reachable ones
    assert int(eng.needed.item()) == r["rect_total"] and r["listed"] < r["rect_total"]
    assert int(eng.status.item()) == 0


def test_render_fwd_matches_oracle(tiny):
    gi = fetch_img(tiny["eng"])
    io = tiny["io"]
    errs, frac = compare_images(gi, io, io["margin"])
    ok = io["margin"] >= FRAGILE
    ranges, ids = fetch_bins(tiny["eng"])
    # median fragment and last contributor name the same surfels
    med_g = np.where(gi["med"] == 0xffffffff, -1, ids[np.minimum(gi["med"], len(ids) - 1)])
    med_o = np.where(io["med"] < 0, -1, tiny["ids"][np.maximum(io["med"], 0)])
    assert np.array_equal(med_g[ok], med_o[ok])
    H, W = gi["alpha"].shape
    tile = (np.arange(H)[:, None] // 16) * ((W + 15) // 16) + np.arange(W)[None, :] // 16
    start_g, start_o = ranges[tile], tiny["off"][tile]
    lg = np.where(gi["last"] > start_g, ids[np.maximum(gi["last"] - 1, 0)], -1)
    lo = np.where(io["last"] > start_o, tiny["ids"][np.maximum(io["last"] - 1, 0)], -1)
    assert np.array_equal(lg[ok], lo[ok])
    # invariants on every pixel
    assert np.all(gi["T"] >= 1e-4 * (1 - 1e-6)) and np.all(gi["T"] <= 1)
    assert np.abs(gi["alpha"] + gi["T"] - 1).max() <= 1e-6


def test_work_counters_match_oracle(tiny):
    eng = tiny["eng"]
    n_eval, n_con, n_bwd = eng.count(tiny["cs"])
    io = tiny["io"]
    # exact when no decision is fragile; allow the fragile pixels' worth of slack
    nfr = int((io["margin"] < FRAGILE).sum())
    assert abs(n_con - io["n_con"]) <= 4 * nfr + 0
    assert abs(n_eval - io["n_eval"]) <= 64 * nfr + 0


def test_loss_matches_oracle(tiny, cuda):
    import torch
    eng = tiny["eng"]
    img = tiny["io"]["rgb"].astype(np.float32)
    tgt = tiny["tgt"]
    lv = eng.loss(torch.from_numpy(tgt).to(cuda)[None], img=torch.from_numpy(img).to(cuda)[None].contiguous())
    torch.cuda.synchronize()
    ref = oracle.ssim_loss(img.astype(np.float64), tgt)
    lv = lv.cpu().numpy()[0]
    assert abs(lv[0] - ref["loss"]) <= 1e-6 * max(1, abs(ref["loss"])) + 2e-7
    assert abs(lv[2] - ref["ssim"]) <= 2e-6
    dt = eng.d_img[0].cpu().numpy()
    ds = eng.d_img_ssim[0].cpu().numpy()
    assert np.abs(dt - ref["d_total"]).max() <= 1e-4 * np.abs(ref["d_total"]).max()
    assert np.abs(ds - ref["d_ssim"]).max() <= 1e-4 * np.abs(ref["d_ssim"]).max()


@pytest.mark.parametrize("W,H", [(150, 37), (64, 16), (65, 17), (1, 1), (64, 45), (65, 46), (3, 200), (300, 2)])
def test_loss_ragged_multi_view(cuda, W, H):
    """Loss strips of 64 columns x 45 rows over sizes that leave partial strips (and a single pixel), two
    views per call (the per-strip sums of both views are kept apart whatever XCD runs each strip)."""
    import torch
    from paper_2411_00771_amd import raster
    rng = np.random.default_rng(W * 100 + H)
    img = rng.uniform(0, 1, (2, 3, H, W)).astype(np.float32)
    tgt = rng.uniform(0, 1, (2, 3, H, W)).astype(np.float32)
    eng = raster.Engine(16, W, H, 2, capacity=1 << 10)
    lv = eng.loss(torch.from_numpy(tgt).to(cuda), img=torch.from_numpy(img).to(cuda)).cpu().numpy()
    dt, ds = eng.d_img.cpu().numpy(), eng.d_img_ssim.cpu().numpy()
    for v in range(2):
        ref = oracle.ssim_loss(img[v].astype(np.float64), tgt[v])
        assert abs(lv[v][0] - ref["loss"]) <= 1e-6 * max(1, abs(ref["loss"])) + 2e-7
        assert abs(lv[v][2] - ref["ssim"]) <= 2e-6
        assert np.abs(dt[v] - ref["d_total"]).max() <= 1e-4 * np.abs(ref["d_total"]).max()
        assert np.abs(ds[v] - ref["d_ssim"]).max() <= 1e-4 * np.abs(ref["d_ssim"]).max()


def _order_bucket(length):
    """Log-scale bucket of a list length (two per octave, 64 buckets), as the launch order defines it."""
    out = np.zeros(length.shape, np.int64)
    nz = length > 0
    e = np.floor(np.log2(np.maximum(length, 1))).astype(np.int64)
    half = np.where(e >= 1, (length >> np.maximum(e - 1, 0)) & 1, 0)
    out[nz] = np.minimum(2 * e[nz] + 1 + half[nz], 63)
    return out


@pytest.mark.parametrize("W,H,views", [(200, 150, 3), (1600, 1066, 1), (1000, 800, 3), (96, 64, 40)])
def test_launch_order_heaviest_first(cuda, W, H, views):
    """The bins' launch order: per chunk of up to 32 views, a permutation of the chunk's tiles (local
    indices) by descending length bucket, ties in index order; rendering is unchanged by it.  Up to
    8192 tiles of at most 32 views the scan and the order share one workgroup (one or several 1024-tile
    rounds); otherwise the multi-workgroup form (above 8192 tiles, or 40 views in two chunks)."""
    import torch
    sc = scenes.tiny_scene(5, 3000)
    dists = np.linspace(2.5, 3.5, views)
    cams = [scenes.tiny_camera(W, H, dist=float(d)) for d in dists]
    eng, _, cs = gpu_forward(sc, cams, capacity=1 << 20)
    torch.cuda.synchronize()
    assert eng.status.item() == 0
    T = eng.tiles
    m = views * T
    ranges = eng.ranges.cpu().numpy().view(np.uint32).astype(np.int64)[: m + 1]
    order = eng.order.cpu().numpy().view(np.uint32).astype(np.int64)[:m]
    length = ranges[1:] - ranges[:-1]
    assert ranges[0] == 0 and np.all(length >= 0) and ranges[-1] <= int(eng.needed.item())
    bk = _order_bucket(length)
    for v0 in range(0, views, 32):
        a, b = v0 * T, min(views, v0 + 32) * T
        ref = np.lexsort((np.arange(b - a), -bk[a:b]))
        assert np.array_equal(order[a:b], ref), v0
    assert len(np.unique(bk)) > 3
    # the same images without the order
    img = eng.rgb.clone()
    eng._bins.order = None
    eng.render(cs)
    torch.cuda.synchronize()
    assert torch.equal(img, eng.rgb)


def _upstream(tiny, seed=3):
    io = tiny["io"]
    H, W = io["alpha"].shape
    rng = np.random.default_rng(seed)
    ok = (io["margin"] >= FRAGILE).astype(np.float64)
    lo = oracle.ssim_loss(io["rgb"], tiny["tgt"])
    up = dict(d_rgb=lo["d_total"] * ok, d_rgb_ssim=lo["d_ssim"] * ok,
              d_depth=rng.normal(size=(H, W)) * 1e-5 * ok, d_depth_med=rng.normal(size=(H, W)) * 1e-5 * ok,
              d_normal=rng.normal(size=(3, H, W)) * 1e-4 * ok, d_alpha=rng.normal(size=(H, W)) * 1e-4 * ok)
    return {k: v.astype(np.float32) for k, v in up.items()}


def test_split_backward_equals_combined(tiny, cuda):
    """cgv2_render_bwd_records followed by cgv2_project_bwd gives what cgv2_render_bwd gives (up to the
    order of float atomics)."""
    import torch
    from paper_2411_00771_amd import raster
    eng, params, cs = tiny["eng"], tiny["params"], tiny["cs"]
    eng.forward(params, cs)
    t = {k: torch.from_numpy(v).to(cuda)[None].contiguous() for k, v in _upstream(tiny, seed=11).items()}
    g1, g2 = raster.Grads(params, 1), raster.Grads(params, 1)
    eng.backward(params, cs, g1, **t)
    eng.backward_records(cs, **t)
    eng.project_backward(params, cs, g2)
    torch.cuda.synchronize()
    for name in ("mean", "log_scale", "quat", "opacity_logit", "sh", "g_view_total", "g_view_ssim"):
        grad_close(name, getattr(g2, name).cpu().numpy(), getattr(g1, name).cpu().numpy(), rel=1e-5)


def test_render_bwd_matches_oracle(tiny, cuda):
    import torch
    from paper_2411_00771_amd import raster
    eng, params, cs = tiny["eng"], tiny["params"], tiny["cs"]
    eng.forward(params, cs)
    up = _upstream(tiny)
    g = raster.Grads(params, 1)
    # the view-space gradients are written whole (zeros outside the view's list): sentinel-filled views
    # at odd float offsets of larger buffers, whose guard elements must stay untouched
    n = params.n
    bufs = [torch.full((2 * n + 8,), 7.0, device=cuda) for _ in range(2)]
    g.g_view_total = bufs[0][1:1 + 2 * n].view(1, 2, n)
    g.g_view_ssim = bufs[1][3:3 + 2 * n].view(1, 2, n)
    t = {k: torch.from_numpy(v).to(cuda)[None].contiguous() for k, v in up.items()}
    eng.backward(params, cs, g, **t)
    torch.cuda.synchronize()
    b0, b1 = bufs[0].cpu().numpy(), bufs[1].cpu().numpy()
    assert np.all(b0[:1] == 7.0) and np.all(b0[1 + 2 * n:] == 7.0)
    assert np.all(b1[:3] == 7.0) and np.all(b1[3 + 2 * n:] == 7.0)
    ref = oracle.backward_view(tiny["sc"], tiny["cam"], tiny["po"], tiny["off"], tiny["ids"],
                               {k: v.astype(np.float64) for k, v in up.items()})
    rp = ref["params"]
    grad_close("mean", g.mean.cpu().numpy(), rp["mean"])
    grad_close("log_scale", g.log_scale.cpu().numpy(), rp["log_scale"])
    grad_close("quat", g.quat.cpu().numpy(), rp["quat"])
    grad_close("opacity_logit", g.opacity_logit.cpu().numpy(), rp["opacity_logit"])
    grad_close("sh", raster.Params.sh_planar(g.sh), rp["sh"])
    grad_close("g_view_total", g.g_view_total[0].cpu().numpy().T, ref["g_total"])
    grad_close("g_view_ssim", g.g_view_ssim[0].cpu().numpy().T, ref["g_ssim"])


def test_densify_matches_oracle(tiny, cuda):
    # densify on the oracle's view-space gradients, visibility and radii of the tiny view, rounded to FP32
    # and given to both sides
    import torch
    from paper_2411_00771_amd import raster
    eng, params, cs = tiny["eng"], tiny["params"], tiny["cs"]
    po = tiny["po"]
    up = _upstream(tiny, seed=5)
    ref = oracle.backward_view(tiny["sc"], tiny["cam"], po, tiny["off"], tiny["ids"],
                               {k: v.astype(np.float64) for k, v in up.items()})
    gt = ref["g_total"].astype(np.float32)
    gs = ref["g_ssim"].astype(np.float32)
    flags = po["flags"].astype(np.uint8)
    radius = po["radius"].astype(np.float32)
    vis = (flags & 1) > 0
    lp = (flags & 32) > 0
    assert vis.sum() > 100 and np.abs(gs[vis]).sum() > 0
    g = raster.Grads(params, 1)
    g.g_view_total[0].copy_(torch.from_numpy(np.ascontiguousarray(gt.T)))
    g.g_view_ssim[0].copy_(torch.from_numpy(np.ascontiguousarray(gs.T)))
    eng.flags.view(-1, params.n)[0].copy_(torch.from_numpy(flags))
    eng.radius.view(-1, params.n)[0].copy_(torch.from_numpy(radius))
    st = raster.DensifyState(params.n)
    ost = oracle.new_densify_state(params.n)
    for call in range(2):
        eng.densify(params, g, st, omega=0.9, eta_min=0.05, grad_threshold=2e-6)
        torch.cuda.synchronize()
        r = oracle.densify_stats(gt.astype(np.float64), gs.astype(np.float64), vis, radius, tiny["sc"].log_scale,
                                 ost, 0.9, 0.05, 2e-6, lowpass=lp)
        assert abs(st.scale[0].item() / r["scale"] - 1) <= 1e-6
        assert np.allclose(st.accum_dgd.cpu().numpy(), ost["accum_dgd"], rtol=1e-5, atol=1e-12)
        assert np.allclose(st.accum_total.cpu().numpy(), ost["accum_total"], rtol=1e-5, atol=1e-12)
        assert np.array_equal(st.denom.cpu().numpy(), ost["denom"])
        assert np.array_equal(st.max_radius.cpu().numpy(), ost["max_radius"].astype(np.float32))
        avg = ost["accum_dgd"] / np.maximum(ost["denom"], 1)
        near = np.abs(avg / 2e-6 - 1) < 1e-4
        m = st.mask.cpu().numpy()
        assert np.array_equal(m[~near], r["mask"][~near])
        c = st.counters.cpu().numpy()
        if not near.any():
            assert np.array_equal(c[:6], r["counters"][:6])
    # the engine's own projection again for the tests that follow
    eng.forward(params, cs)
    torch.cuda.synchronize()


@pytest.mark.parametrize("V", [3, 12])
def test_densify_multi_view_matches_oracle(cuda, V):
    # V views in one call against the oracle applied view after view, on synthetic gradients and masks
    import torch
    from paper_2411_00771_amd import raster
    n = 5000
    sc = scenes.tiny_scene(9, n)
    params = raster.Params.from_scene(sc)
    eng = raster.Engine(n, 64, 64, V, capacity=1 << 12)
    rng = np.random.default_rng(V)
    flags = ((rng.random((V, n)) < 0.6) * 1 + (rng.random((V, n)) < 0.1) * 32).astype(np.uint8)
    radius = rng.uniform(0, 20, (V, n)).astype(np.float32)
    eng.flags.copy_(torch.from_numpy(flags.reshape(-1)))
    eng.radius.copy_(torch.from_numpy(radius.reshape(-1)))
    g = raster.Grads(params, V)
    gt = rng.normal(0, 1e-5, (V, 2, n)).astype(np.float32)
    gs = (rng.normal(0, 3e-6, (V, 2, n)) * rng.uniform(0.2, 1.0, (V, 1, 1))).astype(np.float32)
    g.g_view_total.copy_(torch.from_numpy(gt))
    g.g_view_ssim.copy_(torch.from_numpy(gs))
    st = raster.DensifyState(n, V)
    eng.densify(params, g, st, omega=0.9, eta_min=0.05, grad_threshold=2e-6)
    torch.cuda.synchronize()
    ost = oracle.new_densify_state(n)
    for v in range(V):
        r = oracle.densify_stats(gt[v].T, gs[v].T, (flags[v] & 1) > 0, radius[v], sc.log_scale, ost, 0.9, 0.05, 2e-6,
                                 lowpass=(flags[v] & 32) > 0)
        assert abs(st.scale[v].item() / r["scale"] - 1) <= 1e-6, v
    assert np.allclose(st.accum_dgd.cpu().numpy(), ost["accum_dgd"], rtol=1e-5, atol=1e-12)
    assert np.allclose(st.accum_total.cpu().numpy(), ost["accum_total"], rtol=1e-5, atol=1e-12)
    assert np.array_equal(st.denom.cpu().numpy(), ost["denom"])
    assert np.array_equal(st.max_radius.cpu().numpy(), ost["max_radius"].astype(np.float32))


@pytest.mark.parametrize("views,check", [(3, (0, 1, 2)), (34, (0, 31, 32, 33))])
def test_multi_view_batch_equals_single_views(cuda, views, check):
    # with more than 32 views the calls run in chunks of 32 and the bins hold every view at once
    import torch
    w = scenes.workload(0)
    sc = w["scene"]
    cams = [scenes.tiny_camera(96, 80, dist=float(d)) for d in np.linspace(2.5, 3.5, views)]
    for k, c in enumerate(cams):
        c.R = np.array([[np.cos(0.3 * k), 0, np.sin(0.3 * k)], [0, 1, 0], [-np.sin(0.3 * k), 0, np.cos(0.3 * k)]])
    engb, _, _ = gpu_forward(sc, cams, capacity=1 << 21)
    assert engb.status.item() == 0
    for k in check:
        c = cams[k]
        e1, _, _ = gpu_forward(sc, [c], capacity=1 << 17)
        a, b = fetch_img(engb, k), fetch_img(e1, 0)
        for key in ("rgb", "depth", "depth_med", "normal", "alpha", "T", "med"):
            if key == "med":
                continue
            assert np.array_equal(a[key], b[key]), key
    torch.cuda.synchronize()


def test_empty_and_culled(cuda):
    sc = scenes.tiny_scene(1, 64)
    cam = scenes.tiny_camera(40, 24)
    cam.bg = (0.25, 0.5, 0.75)
    # all behind the camera
    sc.mean[2] -= 10.0
    eng, _, _ = gpu_forward(sc, [cam], capacity=1024)
    P = fetch_proj(eng)
    assert np.all((P["flags"][0] & 2) > 0)
    gi = fetch_img(eng)
    assert int(eng.needed.item()) == 0
    assert np.allclose(gi["rgb"], np.array(cam.bg, np.float32)[:, None, None])
    assert np.all(gi["alpha"] == 0)
    # zero surfels
    sc0 = scenes.tiny_scene(1, 0)
    eng0, _, _ = gpu_forward(sc0, [cam], capacity=16)
    assert int(eng0.needed.item()) == 0
    assert np.allclose(fetch_img(eng0)["rgb"], np.array(cam.bg, np.float32)[:, None, None])
    # NaN parameters are culled, not propagated
    sc2 = scenes.tiny_scene(2, 64)
    sc2.mean[0, :5] = np.nan
    sc2.log_scale[0, 5:8] = np.inf
    eng2, _, _ = gpu_forward(sc2, [cam], capacity=4096)
    P2 = fetch_proj(eng2)
    assert np.all((P2["flags"][0][:8] & 16) > 0)
    assert np.isfinite(fetch_img(eng2)["rgb"]).all()


def test_ragged_image_parity(cuda):
    sc = scenes.tiny_scene(7, 600)
    cam = scenes.tiny_camera(100, 37)
    eng, _, _ = gpu_forward(sc, [cam], capacity=1 << 15)
    po, off, ids, io = oracle.forward_view(sc, cam)
    compare_images(fetch_img(eng), io, io["margin"], max_fragile_frac=2e-3)
    P = fetch_proj(eng)
    ranges, gids = fetch_bins(eng)
    compare_lists(ranges, gids, po, cam, P=P, max_excluded=3)


def test_overflow_reports_needed(cuda):
    import torch
    sc = scenes.tiny_scene(3, 800)
    cam = scenes.tiny_camera(64, 64)
    eng, params, cs = gpu_forward(sc, [cam], capacity=32)
    assert int(eng.status.item()) == 1
    po, off, ids, io = oracle.forward_view(sc, cam)
    K = int(eng.needed.item())
    # the staged entries: every tile of every rect (equal unless a bbox edge sits on a tile boundary)
    assert abs(K - oracle.bin_view(po, cam)[2]["rect_total"]) <= 2
    # render leaves the images untouched while the status is set
    eng.rgb.fill_(float("nan"))
    eng.render(cs)
    torch.cuda.synchronize()
    assert torch.isnan(eng.rgb).all()
    # rerun with the reported capacity
    eng.set_capacity(K)
    eng.status.zero_()
    eng.forward(params, cs)
    torch.cuda.synchronize()
    assert int(eng.status.item()) == 0
    compare_images(fetch_img(eng), io, io["margin"], max_fragile_frac=2e-3)


def test_long_tile_lists_sorted_bit_exact(cuda):
    # 20,000 surfels stacked over one tile: exercises the 16K-entry LDS sort and the global merge
    rng = np.random.default_rng(11)
    n = 20000
    sc = scenes.tiny_scene(4, n)
    sc.mean[0] = rng.uniform(-0.02, 0.02, n).astype(np.float32)
    sc.mean[1] = rng.uniform(-0.02, 0.02, n).astype(np.float32)
    sc.mean[2] = np.round(rng.uniform(-1, 1, n), 2).astype(np.float32)  # many exact depth ties
    sc.log_scale[:] = np.float32(np.log(0.004))
    cam = scenes.tiny_camera(64, 64)
    eng, _, _ = gpu_forward(sc, [cam], capacity=1 << 18)
    P = fetch_proj(eng)
    ranges, ids = fetch_bins(eng)
    assert (np.diff(ranges).max()) > 16384
    compare_lists(ranges, ids, oracle.project(sc, cam), cam, P=P, max_excluded=4)


def test_tile_lists_of_every_sort_class_bit_exact(cuda):
    """Tiles holding exactly L entries for L around every power of two of the per-tile sorts (one wave's
    registers with 1, 2, 4, 8 or 16 keys per lane up to 1024 entries, one 1024-thread workgroup in LDS
    above), with many exact depth ties: the lists equal the oracle's entry for entry."""
    lengths = [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 700, 1024, 1025, 1500, 2048, 2049,
               3000]
    cam = scenes.tiny_camera(96, 64)
    tx = (cam.width + 15) // 16
    rng = np.random.default_rng(23)
    f = float(np.float32(cam.fx))
    mean, tiles_of = [], []
    for t, L in enumerate(lengths):
        ox, oy = (t % tx) * 16, (t // tx) * 16
        z = np.round(rng.uniform(2.0, 4.0, L), 1)  # exact depth ties
        px = ox + rng.uniform(5.0, 11.0, L)
        py = oy + rng.uniform(5.0, 11.0, L)
        mean.append(np.stack([(px - cam.cx) * z / f, (py - cam.cy) * z / f, z - 3.0]))
        tiles_of += [t] * L
    mean = np.concatenate(mean, 1)
    n = mean.shape[1]
    sc = scenes.tiny_scene(23, n)
    sc.mean = mean.astype(np.float32)
    sc.log_scale[:] = np.float32(np.log(0.004))
    sc.quat[:] = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    eng, _, _ = gpu_forward(sc, [cam], capacity=1 << 16)
    assert eng.status.item() == 0
    P = fetch_proj(eng)
    ranges, ids = fetch_bins(eng)
    assert np.array_equal(np.diff(ranges)[:len(lengths)], lengths)
    compare_lists(ranges, ids, oracle.project(sc, cam), cam, P=P, max_excluded=0)


@pytest.mark.parametrize("seed", range(12))
def test_property_scenes_against_oracle(cuda, seed):
    """Seeded random small scenes of the oracle's brute-force property pin, on the GPU: 1-64 surfels of
    scale 0.01-0.6, exact depth ties, a third edge-on, centres off screen, odd image sizes; lists bit-exact
    and images within the tolerance on non-fragile pixels."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 65))
    size = [(16, 16), (33, 17), (48, 40), (70, 23)][seed % 4]
    sc = scenes.tiny_scene(seed, n)
    sc.log_scale[:] = rng.uniform(np.log(0.01), np.log(0.6), size=sc.log_scale.shape).astype(np.float32)
    if seed % 2:
        sc.mean[2] = np.round(sc.mean[2], 1)
        sc.quat[:, : n // 3] = np.array([[0.7071068], [0.7071068], [0.0], [0.0]], np.float32)
    sc.mean[:2] *= np.float32(1.6)
    cam = scenes.tiny_camera(*size)
    eng, _, _ = gpu_forward(sc, [cam], capacity=1 << 14)
    assert eng.status.item() == 0
    po, off, ids, io = oracle.forward_view(sc, cam)
    ranges, gids = fetch_bins(eng)
    compare_lists(ranges, gids, po, cam, P=fetch_proj(eng), max_excluded=4)
    compare_images(fetch_img(eng), io, io["margin"], max_fragile_frac=0.05)


def test_large_rects_staged_in_chunks_bit_exact(cuda):
    """Surfels whose rect covers far more than the 256 tiles a staging group takes itself (the rest goes
    through the 128-tile chunk queue), among ordinary ones: the lists equal the oracle's entry for entry
    and the images match it."""
    rng = np.random.default_rng(31)
    sc = scenes.tiny_scene(31, 3000)
    cam = scenes.tiny_camera(480, 400)
    # 24 wide surfels close to the camera, some elongated, at random orientations
    k = 24
    sc.mean[:, :k] = np.stack([rng.uniform(-0.6, 0.6, k), rng.uniform(-0.5, 0.5, k),
                               rng.uniform(1.5, 2.4, k)]).astype(np.float32)
    sc.log_scale[0, :k] = np.log(rng.uniform(0.5, 1.2, k)).astype(np.float32)
    sc.log_scale[1, :k] = np.log(rng.uniform(0.05, 1.2, k)).astype(np.float32)
    po = oracle.project(sc, cam)
    tr = po["tile_rect"].astype(np.int64)
    tiles = (tr[:, 2] - tr[:, 0]) * (tr[:, 3] - tr[:, 1])
    assert (tiles > 256).sum() >= 10 and tiles.max() > 2 * 256  # several rects need queued chunks
    eng, _, _ = gpu_forward(sc, [cam], capacity=1 << 19)
    P = fetch_proj(eng)
    ranges, ids = fetch_bins(eng)
    r = compare_lists(ranges, ids, po, cam, P=P, max_excluded=8)
    assert r["surfels"] <= 2
    assert int(eng.needed.item()) == r["rect_total"]
    assert int(eng.status.item()) == 0
    off, oids, _ = oracle.bin_view(po, cam)
    io = oracle.render(po, cam, off, oids)
    compare_images(fetch_img(eng), io, io["margin"], max_fragile_frac=5e-3)


def test_zero_grads_clears_exactly_the_parameter_gradients(cuda):
    """cgv2_zero_grads: the five parameter-gradient arrays zeroed whatever their alignment and length (arrays
    placed at odd float offsets, lengths not multiples of 4, for SH degrees 0-3), nothing before or after
    them touched, the view-space gradients left as they were."""
    import ctypes
    import torch
    from paper_2411_00771_amd import _lib
    L = _lib.lib()
    for deg, n in ((0, 1), (1, 7), (2, 1001), (3, 65537)):
        K = (deg + 1) ** 2
        counts = [3 * n, 2 * n, 4 * n, n, 3 * K * n]
        total = sum(c + 9 for c in counts) + 8
        buf = torch.full((total,), 7.0, device="cuda")
        offs, o = [], 1
        for c in counts:
            offs.append(o)
            o += c + 9
        gv = torch.full((2, 2, n), 5.0, device="cuda")
        g = _lib.Grads(*[ctypes.c_void_p(buf.data_ptr() + 4 * a) for a in offs],
                       ctypes.c_void_p(gv.data_ptr()), ctypes.c_void_p(gv[1].data_ptr()))
        assert L.cgv2_zero_grads(ctypes.byref(g), n, deg, None) == 0
        torch.cuda.synchronize()
        want = torch.full((total,), 7.0, device="cuda")
        for a, c in zip(offs, counts):
            want[a:a + c] = 0.0
        assert torch.equal(buf, want), (deg, n)
        assert bool((gv == 5.0).all())


def test_zeroing_on_a_second_stream_matches_in_line(cuda):
    """The benchmark's step order: the parameter gradients zeroed on a second stream that waits for an event
    after the previous step's chain and is waited for before this step's chain; three steps on three views
    give the same gradients as the same steps with the zeroing in line (each step's chain adds into freshly
    zeroed gradients either way), up to the rounding order of the reverse pass's float atomics."""
    import torch
    from paper_2411_00771_amd import raster
    w = scenes.workload(0)
    sc = w["scene"]
    cams = [scenes.tiny_camera(128, 128, dist=d) for d in (2.8, 3.0, 3.3)]
    params = raster.Params.from_scene(sc)
    eng = raster.Engine(sc.n, 128, 128, 1, capacity=1 << 16)
    tgt = torch.from_numpy(np.ascontiguousarray(w["targets"][0], np.float32)).cuda()[None]

    def run(overlap):
        g = raster.Grads(params, 1)
        out = []
        zs = torch.cuda.Stream()
        free, zeroed = torch.cuda.Event(), torch.cuda.Event()
        free.record()
        for cam in cams:
            cs = eng.cams([cam])
            if overlap:
                zs.wait_event(free)
                with torch.cuda.stream(zs):
                    g.zero_()
                    zeroed.record(zs)
            else:
                g.zero_()
            eng.status.zero_()
            eng.project(params, cs)
            eng.bin_sort(cs)
            eng.render(cs)
            eng.loss(tgt)
            eng.backward_records(cs, d_rgb=eng.d_img, d_rgb_ssim=eng.d_img_ssim)
            if overlap:
                torch.cuda.current_stream().wait_event(zeroed)
            eng.project_backward(params, cs, g)
            if overlap:
                free.record()
            out.append(torch.cat([t.reshape(-1) for t in (g.mean, g.log_scale, g.quat, g.opacity_logit, g.sh)]))
            out[-1] = out[-1].clone()
        torch.cuda.synchronize()
        assert eng.status.item() == 0
        return out

    a, b = run(False), run(True)
    for x, y in zip(a, b):
        # the reverse pass adds with float atomics, so compare to the atomics' rounding, not bit for bit
        assert torch.allclose(x, y, rtol=1e-5, atol=1e-9)
        assert bool((x != 0).any())

