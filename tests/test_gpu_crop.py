"""Visibility-frequency crop volume (Sec. 4) on the GPU against the oracle.

Counts are integers: bit-exact for every point whose decisions are not fragile in the oracle's FP64
margin sense (a decision quantity within 1e-9 relative of its threshold, where an FP64 evaluation in
another order may decide the other way), and within the number of fragile views otherwise.  The
keep mask and the kept count are bit-exact; the ground coordinates and the height range are FP64
values evaluated in a different order: within 1e-12 relative."""
import numpy as np
import pytest

from oracle import visibility as ovis
from paper_2411_00771_amd import scenes

pytestmark = pytest.mark.gpu


def _gpu_counts(P, cams, rho, rf, order=None):
    import torch
    from paper_2411_00771_amd import crop
    Q = P if order is None else P[:, order]
    pt = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).cuda()
    c = crop.visibility_count(pt, cams, rho, rf)
    torch.cuda.synchronize()
    got = c.cpu().numpy().view(np.uint32).astype(np.int64)
    if order is not None:
        back = np.empty_like(got)
        back[order] = got
        got = back
    return got


def _check_counts(P, cams, rho, rf, order=None):
    print(f"[crop] m={P.shape[1]} V={len(cams)} rho={rho} rf={rf} order={'given' if order is None else 'permuted'}",
          flush=True)
    ref, frag = ovis.visibility_count(P, cams, rho, rf)
    got = _gpu_counts(P, cams, rho, rf, order)
    ok = frag == 0
    assert np.array_equal(got[ok], ref[ok]), int((got[ok] != ref[ok]).sum())
    assert np.all(np.abs(got - ref) <= frag)
    return ref


def _small_city(n=20000, views=24, W=320, H=240, seed=3, L=300.0):
    city = scenes.make_city(seed, L=L, n_boxes=20)
    P = scenes.city_points(seed + 1, n, city)
    cams = scenes.aerial_cameras(seed + 2, city, count=views, width=W, height=H, alt=(30.0, 90.0))
    return city, P, cams


@pytest.mark.parametrize("rf", [2.1213, 0.5, 0.3])
def test_counts_small_city_orders(cuda, rf):
    _, P, cams = _small_city()
    ref = _check_counts(P, cams, 0.4, rf)
    assert 0 < ref.mean() < len(cams)
    # the same counts in Morton order (small workgroup boxes) and in a random order (large boxes)
    _check_counts(P, cams, 0.4, rf, order=scenes.morton_order(P))
    _check_counts(P, cams, 0.4, rf, order=np.random.default_rng(1).permutation(P.shape[1]))


@pytest.mark.parametrize("m", [0, 1, 1023, 1024, 1025, 5000])
def test_counts_ragged_sizes(cuda, m):
    _, P, cams = _small_city(n=max(m, 1), views=7)
    P = P[:, :m]
    if m == 0:
        assert _gpu_counts(P, cams, 0.4, 2.0).size == 0
        return
    _check_counts(P, cams, 0.4, 2.0)


def test_counts_many_views_and_near_cases(cuda):
    """More views than one classification pass (256) and more than one launch (4096); points behind the
    cameras, before znear and within the sphere radius of the camera plane."""
    rng = np.random.default_rng(7)
    cams = []
    for k in range(4200):
        c = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-2, 2)])
        yaw, pitch = rng.uniform(0, 2 * np.pi), rng.uniform(-0.5, 0.5)
        fwd = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
        right = np.cross(fwd, [0.0, 0.0, 1.0])
        cams.append(scenes._look_camera(c, fwd, right, 64, 48, 70.0))
    P = rng.uniform(-6, 6, (3, 300)).astype(np.float32)
    P[2] *= 0.3
    ref = _check_counts(P, cams, 0.8, 1.0)
    assert ref.min() >= 0 and ref.max() > 0
    _check_counts(P, cams, 0.8, 0.25)


def test_crop_volume_matches_oracle(cuda):
    import torch
    from paper_2411_00771_amd import crop
    _, P, cams = _small_city(n=30011)
    cnt = _check_counts(P, cams, 0.4, 2.1213)
    pt = torch.from_numpy(P).cuda()
    ct = torch.from_numpy(cnt.astype(np.int32)).cuda()
    c, s = np.cos(0.3), np.sin(0.3)
    for T in (np.hstack([np.eye(3), np.zeros((3, 1))]),
              np.array([[c, -s, 0, 5.0], [s, c, 0, -2.0], [0, 0, 1.0, -10.0]])):
        for tau in (0, 3, int(cnt.max()), int(cnt.max()) + 1):
            keep, ground, (h0, h1) = crop.crop_volume(pt, ct, tau, T)
            rk, rg, rh0, rh1 = ovis.crop_volume(P, cnt, tau, T)
            assert np.array_equal(keep.cpu().numpy().astype(bool), rk)
            g = ground.cpu().numpy()
            assert g.shape == rg.shape
            assert np.allclose(g, rg, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(rg).max() if rg.size else 1.0))
            if rk.any():
                assert np.isclose(h0, rh0, rtol=1e-12, atol=1e-12) and np.isclose(h1, rh1, rtol=1e-12, atol=1e-12)
            else:
                assert np.isnan(h0) and np.isnan(h1)


def test_crop_full_size_sampled(cuda):
    """The 1.47 km^2, 958-view, 31.4 M-point workload at 1920x1080: counts of 20,000 sampled points
    against the oracle over all views, and properties over all points."""
    import torch
    from paper_2411_00771_amd import crop
    w = scenes.crop_workload()
    P, cams = w["points"], w["cameras"]
    m = P.shape[1]
    rho, rf = 0.8, 2.1213
    pt = torch.from_numpy(P).cuda()
    cnt = crop.visibility_count(pt, cams, rho, rf)
    torch.cuda.synchronize()
    got = cnt.cpu().numpy().view(np.uint32).astype(np.int64)
    assert got.max() <= len(cams)
    idx = np.random.default_rng(11).choice(m, 20000, replace=False)
    ref, frag = ovis.visibility_count(P[:, idx], cams, rho, rf)
    ok = frag == 0
    assert np.array_equal(got[idx][ok], ref[ok])
    assert np.all(np.abs(got[idx] - ref) <= frag)
    keep, ground, (h0, h1) = crop.crop_volume(pt, cnt, 3, np.hstack([np.eye(3), np.zeros((3, 1))]))
    kp = keep.cpu().numpy().astype(bool)
    assert np.array_equal(kp, got >= 3)
    assert ground.shape[1] == kp.sum()
    assert h0 == float(P[2, kp].astype(np.float64).min()) and h1 == float(P[2, kp].astype(np.float64).max())
