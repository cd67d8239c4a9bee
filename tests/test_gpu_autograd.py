"""Differentiation form: Rasterize2DGS / L1SSIMLoss as torch.autograd Functions.

A 512-surfel crop of the aerial generator (the surfels nearest a ground point) in a 64x64 window:
autograd gradients vs the oracle's analytic gradients and vs FP64 central differences (eps 1e-4) of
the oracle's loss; 8- and 34-view launches equal the sum of single-view launches; nothing per fragment
is saved for the backward."""
import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes
from tests.helpers import FRAGILE, grad_close

pytestmark = pytest.mark.gpu


def _crop_and_cams(n_views=8):
    city = scenes.make_city(2, L=400.0, n_boxes=10)
    sc_full = scenes.city_scene(2, 60_000, L=400.0, city=city)
    c0 = np.array([10.0, -20.0, float(city.height(np.array([10.0]), np.array([-20.0]))[0])])
    d = np.linalg.norm(sc_full.mean.T.astype(np.float64) - c0, axis=1)
    sc = sc_full.subset(np.sort(np.argsort(d)[:512]))
    cams = []
    rng = np.random.default_rng(3)
    for k in range(n_views):
        off = rng.normal(size=2) * 3.0
        pos = c0 + np.array([off[0], off[1], 25.0 + 3 * k])
        fwd = c0 - pos
        cams.append(scenes._look_camera(pos, fwd, np.array([1.0, 0.0, 0.0]), 64, 64, 50.0))
    return sc, cams


def _autograd_grads(sc, cams, targets, cuda):
    import torch
    from paper_2411_00771_amd import raster
    eng = raster.Engine(sc.n, 64, 64, len(cams), capacity=1 << 18)
    cs = eng.cams(cams)
    # the SH block of each surfel is contiguous on the device: [n][K][3]
    ts = [torch.from_numpy(getattr(sc, k)).to(cuda).requires_grad_(True)
          for k in ("mean", "log_scale", "quat", "opacity_logit")]
    ts.append(torch.from_numpy(np.ascontiguousarray(sc.sh.transpose(2, 0, 1))).to(cuda).requires_grad_(True))
    seen = []
    orig = eng.backward

    def spy(*a, **kw):
        seen.append(sorted(k for k, v in kw.items() if v is not None))
        return orig(*a, **kw)

    eng.backward = spy
    rgb, depth, dmed, normal, alpha = raster.rasterize(ts, eng, cs, sc.sh_degree)
    loss = raster.L1SSIMLoss.apply(rgb, torch.from_numpy(np.stack(targets)).to(cuda), eng, 0.2)
    loss.backward()
    torch.cuda.synchronize()
    assert eng.status.item() == 0
    # only the colour terms reach the reverse pass (unused outputs are not materialized as zeros)
    assert seen == [["d_rgb", "d_rgb_ssim"]]
    grads = [t.grad.cpu().numpy() for t in ts[:4]] + [raster.Params.sh_planar(ts[4].grad)]
    return eng, grads, loss.item()


def test_autograd_matches_oracle_and_fd(cuda):
    sc, cams = _crop_and_cams(1)
    cam = cams[0]
    tgt = scenes.random_target(7, 64, 64)
    eng, g, lval = _autograd_grads(sc, [cam], [tgt], cuda)
    # oracle analytic gradient on the same loss
    P = oracle._scene64(sc)
    proj, off, ids, img = oracle.forward_view(P, cam)
    assert (img["margin"] < FRAGILE).mean() <= 5e-3
    lo = oracle.ssim_loss(img["rgb"], tgt)
    assert abs(lval - lo["loss"]) <= 1e-5 * lo["loss"]
    ref = oracle.backward_view(P, cam, proj, off, ids, dict(d_rgb=lo["d_total"]))["params"]
    names = ("mean", "log_scale", "quat", "opacity_logit", "sh")
    for name, gg in zip(names, g):
        grad_close(name, gg, ref[name])
    # FP64 central differences of the oracle loss, eps = 1e-4, on parameters drawn among those whose gradient
    # is not negligible (|g| >= 0.1 rms of the group) until 8 per group keep every discrete decision at +-eps
    rng = np.random.default_rng(0)
    eps = 1e-4
    sig0 = img["sig"]
    for name, gg in zip(names, g):
        flat = P[name].reshape(-1)
        r = ref[name].reshape(-1)
        cand = np.flatnonzero(np.abs(r) >= 0.1 * np.sqrt(np.mean(r ** 2)))
        fd, an, orc = [], [], []
        for i in rng.permutation(cand)[:60]:
            vals = []
            for sgn in (1, -1):
                Q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in P.items()}
                Q[name].reshape(-1)[i] += sgn * eps
                _, _, _, im2 = oracle.forward_view(Q, cam)
                vals.append((oracle.ssim_loss(im2["rgb"], tgt)["loss"], im2["sig"]))
            if not (np.array_equal(vals[0][1], sig0) and np.array_equal(vals[1][1], sig0)):
                continue
            fd.append((vals[0][0] - vals[1][0]) / (2 * eps))
            an.append(gg.reshape(-1)[i])
            orc.append(r[i])
            if len(fd) == 8:
                break
        fd, an, orc = np.array(fd), np.array(an), np.array(orc)
        assert len(fd) == 8, f"{name}: only {len(fd)} usable finite-difference samples"
        e_gpu = np.linalg.norm(fd - an) / np.linalg.norm(fd)
        e_orc = np.linalg.norm(fd - orc) / np.linalg.norm(fd)
        print(f"[fd] {name}: GPU vs FD {e_gpu:.2e}, oracle vs FD {e_orc:.2e}", flush=True)
        assert e_orc <= 1e-5, name
        assert e_gpu <= 1e-3, name


@pytest.mark.parametrize("V", [8, 34])
def test_batched_views_equal_sum_of_single_views(cuda, V):
    # 34 views: every call runs in chunks of 32 views
    sc, cams = _crop_and_cams(V)
    tg = [scenes.random_target(20 + k, 64, 64) for k in range(V)]
    eng8, g8, l8 = _autograd_grads(sc, cams, tg, cuda)
    acc = [np.zeros_like(x) for x in g8]
    ltot = 0.0
    for k in range(V):
        _, g1, l1 = _autograd_grads(sc, [cams[k]], [tg[k]], cuda)
        for a, b in zip(acc, g1):
            a += b
        ltot += l1
    assert abs(l8 - ltot) <= 1e-5 * abs(ltot)
    for name, a, b in zip(("mean", "log_scale", "quat", "opacity_logit", "sh"), g8, acc):
        grad_close(name, a, b, rel=1e-4)
    # the only state kept for the backward is the per-pixel checkpoint (12 B / pixel) + bins
    assert eng8.T_final.element_size() * eng8.T_final.numel() == 4 * V * 64 * 64


def test_backward_refuses_stale_or_overflowed_state(cuda):
    """The autograd outputs alias the engine's buffers: a backward after a second forward on the same engine
    raises instead of reading that forward's checkpoint, and so does a backward after an overflow."""
    import torch
    from paper_2411_00771_amd import raster
    sc, cams = _crop_and_cams(1)
    tgt = torch.from_numpy(scenes.random_target(7, 64, 64)[None]).to(cuda)

    def leaves():
        ts = [torch.from_numpy(getattr(sc, k)).to(cuda).requires_grad_(True)
              for k in ("mean", "log_scale", "quat", "opacity_logit")]
        ts.append(torch.from_numpy(np.ascontiguousarray(sc.sh.transpose(2, 0, 1))).to(cuda).requires_grad_(True))
        return ts

    eng = raster.Engine(sc.n, 64, 64, 1, capacity=1 << 18)
    cs = eng.cams(cams)
    out1 = raster.rasterize(leaves(), eng, cs, sc.sh_degree)
    loss1 = raster.L1SSIMLoss.apply(out1[0], tgt, eng, 0.2)
    out2 = raster.rasterize(leaves(), eng, cs, sc.sh_degree)
    with pytest.raises(RuntimeError, match="another"):
        loss1.backward()
    # the latest graph still works
    loss2 = raster.L1SSIMLoss.apply(out2[0], tgt, eng, 0.2)
    loss2.backward()
    torch.cuda.synchronize()
    small = raster.Engine(sc.n, 64, 64, 1, capacity=16)
    small.status.zero_()
    out3 = raster.rasterize(leaves(), small, small.cams(cams), sc.sh_degree)
    loss3 = raster.L1SSIMLoss.apply(out3[0], tgt, small, 0.2)
    with pytest.raises(RuntimeError, match="overflowed"):
        loss3.backward()
