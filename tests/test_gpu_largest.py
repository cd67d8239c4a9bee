"""The largest case: 10 M surfels (log-normal scales, 10 % degenerate elongated), one 8-view 1600x1066
training step interleaved with served 3840x2160 depth/normal renders of 64 nadir mesh-extraction
views, on one GPU.

Checks: (1) the mix changes nothing: every served render that is also rendered alone is bit-identical,
the training loss is bit-identical and the gradients agree to float-atomic ordering; (2) parity with
the oracle at this size on one training view and one 4K served view: tile lists bit-exact, images on
sampled tiles the oracle renders one by one (lists bit-exact but for counted rounding ties of the
projection and fragile reach decisions)."""
import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes
from tests.helpers import compare_lists, compare_sampled_tiles, fetch_bins, grad_close

pytestmark = pytest.mark.gpu

SERVE_CHECK = (0, 27, 63)  # served views also rendered alone


@pytest.fixture(scope="module")
def largest(cuda):
    import torch
    from paper_2411_00771_amd import raster, server
    w = scenes.workload(4)
    sc = w["scene"]
    print(f"[largest] {w['name']}: n={sc.n}", flush=True)
    params = raster.Params.from_scene(sc)
    cams = w["cameras"]
    serve_cams = w["serve_cameras"]
    eng = raster.Engine(sc.n, cams[0].width, cams[0].height, len(cams), capacity=1 << 20)
    cs = eng.cams(cams)
    eng.fit_capacity(params, cs)
    targets = torch.stack([torch.from_numpy(scenes.random_target(400 + i, c.width, c.height)) for i, c in
                           enumerate(cams)]).to(cuda)

    def train_step():
        g = raster.Grads(params, len(cams))
        st = raster.DensifyState(sc.n, len(cams))
        eng.forward(params, cs)
        lv = eng.loss(targets).clone()
        eng.backward(params, cs, g, d_rgb=eng.d_img, d_rgb_ssim=eng.d_img_ssim)
        eng.densify(params, g, st)
        return lv, g, st

    # alone: the training step, then the checked served views one at a time
    lv0, g0, st0 = train_step()
    torch.cuda.synchronize()
    assert eng.status.item() == 0
    srv = server.Server(params, max_slots=4, arena_bytes=64 << 30, intersections_per_pixel=3.0)
    alone = {}
    for k in SERVE_CHECK:
        r = srv.render_alone(serve_cams[k])
        assert r.error is None
        alone[k] = {n: t.clone() for n, t in r.result.items()}
    print("[largest] alone runs done", flush=True)

    # mixed: all 64 served views queued, the training step on its own stream, the server admitting
    # requests while the step runs
    reqs = [srv.submit(c) for c in serve_cams]
    srv.poll()
    ts = torch.cuda.Stream()
    with torch.cuda.stream(ts):
        lv1, g1, st1 = train_step()
    srv.drain()
    torch.cuda.synchronize()
    assert eng.status.item() == 0
    print("[largest] mixed run done", flush=True)
    return dict(sc=sc, params=params, cams=cams, serve_cams=serve_cams, eng=eng, cs=cs, alone=alone, reqs=reqs,
                run0=(lv0, g0, st0), run1=(lv1, g1, st1), srv=srv)


def test_mix_equals_alone(largest):
    reqs = largest["reqs"]
    assert all(r.error is None for r in reqs)
    assert all(r.done for r in reqs)
    for k, ref in largest["alone"].items():
        for name, t in ref.items():
            assert reqs[k].result[name].shape == t.shape
            assert bool((reqs[k].result[name] == t).all()), (k, name)
    (lv0, g0, st0), (lv1, g1, st1) = largest["run0"], largest["run1"]
    # the forward and the loss are deterministic; the gradients are sums of float atomics
    assert bool((lv0 == lv1).all())
    # Two runs differ only in the order of float atomics: the group norms agree to 1e-4, and elementwise
    # to the gradient tolerance (elements with heavy cancellation drift by more than 1e-4 relative; a lost
    # or duplicated update would move an element by a whole term).
    for name in ("mean", "log_scale", "quat", "opacity_logit", "sh", "g_view_total", "g_view_ssim"):
        a, b = getattr(g1, name).cpu().numpy().astype(np.float64), getattr(g0, name).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b), name
        grad_close(name, a, b)
    s0, s1 = st0.scale.cpu().numpy(), st1.scale.cpu().numpy()
    assert np.allclose(s0, s1, rtol=1e-4, atol=0)
    # masks may differ only for surfels at the threshold; count those at most 1e-5 of n
    m0, m1 = st0.mask.cpu().numpy(), st1.mask.cpu().numpy()
    assert np.count_nonzero(m0 != m1) <= max(4, int(1e-5 * m0.size))


def _sample_tiles(ranges, k, seed):
    rng = np.random.default_rng(seed)
    lens = np.diff(ranges)
    longest = np.argsort(lens)[-6:]
    nz = np.flatnonzero(lens)
    pick = rng.choice(nz, size=min(k, len(nz)), replace=False)
    return np.unique(np.concatenate([pick, longest])).astype(np.int32)


def _check_view(sc, cam, eng, v):
    """Bins bit-exact, projection agreement and every output on sampled tiles against the oracle."""
    V, n, T = eng.V, eng.n, eng.tiles
    depth_key = eng.rec.view(V, n, 24)[v, :, 11].cpu().numpy().astype(np.float32)
    rect = eng.rect.view(V, n, 4)[v].cpu().numpy().view(np.uint16).astype(np.int32)
    flags = eng.flags.view(V, n)[v].cpu().numpy().astype(np.int32)
    ranges_all, ids_all = fetch_bins(eng)
    r = ranges_all[v * T:(v + 1) * T + 1]
    ranges, ids = r - r[0], ids_all[int(r[0]):int(r[-1])]
    po = oracle.project(sc, cam)
    P = dict(flags=flags[None], rect=rect[None], rec=np.zeros((1, len(flags), 24), np.float32))
    P["rec"][0, :, 11] = depth_key
    lr = compare_lists(ranges, ids, po, cam, P=P)
    print(f"[largest] lists {lr}", flush=True)
    assert lr["surfels"] <= 32 and lr["fragile_pairs"] <= 5e-4 * lr["listed"]
    vis_o = (po["flags"] & 1) > 0
    vis_g = (flags & 1) > 0
    assert np.mean(vis_o != vis_g) < 1e-5
    both = vis_o & vis_g
    assert np.count_nonzero(depth_key[both].view(np.uint32) != po["depth32"][both].view(np.uint32)) <= \
        max(2, int(1e-6 * both.sum()))
    off, oids, _ = oracle.bin_view(po, cam)
    tiles = _sample_tiles(ranges, 40, 7)
    ref, _, _ = oracle.render_tiles(po, cam, off, oids, tiles)
    worst, fragile, total = compare_sampled_tiles(eng, ref, tiles, v=v)
    print(f"[largest] view {v} of {V}: worst {worst}, fragile {fragile} of {total} pixels", flush=True)
    # 10 % of these surfels are degenerate (axis ratio up to 1000): their intersections are ill-conditioned,
    # so more decisions fall inside the FP32 error bound than on the 1 M scene (0.55 % measured)
    assert fragile <= 1e-2 * total, (fragile, total)


def test_training_view_parity_at_10m(largest):
    _check_view(largest["sc"], largest["cams"][5], largest["eng"], 5)


def test_served_4k_view_parity_at_10m(largest, cuda):
    import torch
    from paper_2411_00771_amd import raster
    sc, params = largest["sc"], largest["params"]
    cam = largest["serve_cams"][27]
    e = raster.Engine(sc.n, cam.width, cam.height, 1, capacity=1 << 20, backward=False)
    cs = e.cams([cam])
    e.fit_capacity(params, cs)
    e.forward(params, cs)
    torch.cuda.synchronize()
    assert e.status.item() == 0
    # the served result (taken in the mix) equals this render bit for bit
    res = largest["reqs"][27].result
    assert bool((res["depth"] == e.depth[0]).all()) and bool((res["normal"] == e.normal[0]).all())
    _check_view(sc, cam, e, 0)
