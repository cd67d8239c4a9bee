"""Pins of the FP64 oracle to facts the paper and the mathematics fix (no GPU).

P1  single camera-facing isotropic surfel: alpha = o exp(-r^2 / 2) in plane units (Eq. 1), depth 3,
    normal flipped towards the camera; below the filter threshold the screen Gaussian takes over
P2  stacked surfels through one pixel centre: T = .05, .0025, 1.25e-4, the fourth excluded
P3  the 0.99 clamp, the 1/255 skip and the opacity cull
P4  per-pixel invariants
P5  tiled render == brute force over all surfels (exact in FP64), incl. property-based scenes
P6  per-tile order == numpy lexsort on (tile, fp32 depth bits, id)
P7  conic bounding box contains and touches the mapped cutoff circle
P8  SH orthonormality by exact quadrature; textbook closed forms of degrees 0-3
P9  analytic gradients == FP64 central differences
P10 view-space gradient == derivative w.r.t. a rigid screen translation of M
P11 DGD (Eq. 2) hand example, clamp at 1, invariance to invisible surfels; elongation rate
P12 SSIM identities, constant-image closed form, finite differences of the loss
P13 contribution (Eq. 3): closed forms for one facing surfel and for two stacked facing surfels;
    tiled == brute force; sum of |P| == the render's contributing pairs
P14 Eq. 4 average and the trimming bound on hand-worked arrays
P15 densification action on a hand-worked six-surfel set: keep, clone, split (identity and quarter-turn
    rotations), trimmed and low-opacity removal, output order and counts
P16 visibility frequency (Sec. 4 crop volume): the sphere-image box in closed form on the axis and
    against dense silhouette sampling off the axis; hand-placed visible / hidden points (behind the
    camera, between two pixel samples, off the image edge); counts as sums over views; the crop
    threshold, height range and ground coordinates under two transforms
P18 the list rule (tile reach): a facing isotropic surfel keeps exactly the tiles within its cutoff
    radius (closed form); on scenes of elongated, tilted surfels no tile with a pixel sample inside the
    cutoff region is dropped (brute force over every sample), while most rect tiles outside it are;
    images from the reach lists equal those from the plain rect lists and the brute-force render
P17 serving storage: float16 rounding at known values, the importance partition, the nearest codeword
    against explicit loops and by construction (ties to the smaller index), the Lloyd update by hand
    (an empty codeword kept), the non-increasing k-means error, and decode(pack) within float16 rounding
"""
import math

import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes

F_VIS = oracle.F_VISIBLE


def one_surfel_scene(mu, scale, logit, q=(1.0, 0.0, 0.0, 0.0), dc=1.0, ls2=None):
    n = len(mu)
    mean = np.array(mu, np.float64).T.reshape(3, n)
    ls = np.full((2, n), math.log(scale)) if ls2 is None else np.array(ls2, np.float64).reshape(2, n)
    quat = np.tile(np.array(q, np.float64).reshape(4, 1), (1, n))
    lg = np.broadcast_to(np.array(logit, np.float64), (n,)).copy()
    sh = np.zeros((16, 3, n))
    sh[0] = dc
    return dict(mean=mean, log_scale=ls, quat=quat, opacity_logit=lg, sh=sh, sh_degree=3)


def f32(v):
    return float(np.float32(v))


def render(P, cam):
    proj = oracle.project(P, cam)
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    return proj, oracle.render(proj, cam, off, ids)


@pytest.mark.parametrize("scale", [0.05, 0.3])
def test_p1_single_facing_surfel_3d_branch(scale):
    cam = scenes.tiny_camera()
    logit = 1.3
    o = 1 / (1 + math.exp(-logit))
    P = one_surfel_scene([(0.0, 0.0, 0.0)], scale, logit)
    proj, img = render(P, cam)
    H, W = cam.height, cam.width
    i = np.arange(W)[None, :] + 0.5
    j = np.arange(H)[:, None] + 0.5
    X = (i - f32(cam.cx)) * 3.0 / f32(cam.fx)
    Y = (j - f32(cam.cy)) * 3.0 / f32(cam.fy)
    a = np.minimum(0.99, o * np.exp(-(X ** 2 + Y ** 2) / (2 * scale ** 2)))
    a = np.where(a < 1 / 255, 0.0, a)
    c = 0.5 + 1.0 / (2 * math.sqrt(math.pi))
    assert np.abs(img["alpha"] - a).max() < 1e-12
    assert np.abs(img["rgb"] - c * a[None]).max() < 1e-12
    assert np.abs(img["depth"] - 3 * a).max() < 1e-12
    assert np.abs(img["depth_med"] - np.where(a > 0, 3.0, 0.0)).max() < 1e-12
    assert np.abs(img["normal"][2] + a).max() < 1e-12 and np.abs(img["normal"][:2]).max() < 1e-15


def test_p1_subpixel_surfel_filter_branch():
    cam = scenes.tiny_camera()
    scale = 0.01  # below 3 / (sqrt(2) f) = 0.0191: the screen filter wins at every sample
    logit = 2.0
    o = 1 / (1 + math.exp(-logit))
    P = one_surfel_scene([(0.0, 0.0, 0.0)], scale, logit)
    proj, img = render(P, cam)
    assert proj["flags"][0] & oracle.F_LOWPASS
    i = np.arange(cam.width)[None, :] + 0.5
    j = np.arange(cam.height)[:, None] + 0.5
    r2 = (i - f32(cam.cx)) ** 2 + (j - f32(cam.cy)) ** 2
    a = np.minimum(0.99, o * np.exp(-r2))
    a = np.where(a < 1 / 255, 0.0, a)
    assert np.abs(img["alpha"] - a).max() < 1e-12
    # the filter branch takes the centre depth
    assert np.abs(img["depth"] - 3 * a).max() < 1e-12


def test_p2_stacked_surfels_stop_rule():
    cam = scenes.tiny_camera()
    px, py = 70, 60
    x, y = px + 0.5, py + 0.5
    zs = [1.0, 1.5, 2.0, 2.5]
    mu = [((x - f32(cam.cx)) * z / f32(cam.fx), (y - f32(cam.cy)) * z / f32(cam.fy), z - 3.0) for z in zs]
    logit = math.log(0.95 / 0.05)
    dcs = np.array([0.1, 0.4, 0.7, 1.0])
    P = one_surfel_scene(mu, 0.2, logit)
    P["sh"][0] = dcs[None, :]
    proj, img = render(P, cam)
    assert abs(img["T"][py, px] - 1.25e-4) < 1e-15
    cols = 0.5 + dcs / (2 * math.sqrt(math.pi))
    expect = sum(cols[k] * 0.95 * 0.05 ** k for k in range(3))
    assert abs(img["rgb"][0, py, px] - expect) < 1e-12
    assert abs(img["depth_med"][py, px] - 1.0) < 1e-12
    assert abs(img["alpha"][py, px] - (1 - 1.25e-4)) < 1e-15
    # three contributors: 'last' is one past the third list entry of that tile
    t = (py // 16) * 8 + px // 16
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    assert list(ids[off[t]:off[t + 1]][:4]) == [0, 1, 2, 3]
    assert img["last"][py, px] == off[t] + 3


def test_p3_clamp_skip_and_cull():
    cam = scenes.tiny_camera()
    px, py = 40, 80
    x, y = px + 0.5, py + 0.5
    pos = lambda z: ((x - f32(cam.cx)) * z / f32(cam.fx), (y - f32(cam.cy)) * z / f32(cam.fy), z - 3.0)
    for o, expect in ((1 - 1e-9, 0.99), (0.0045, 0.0045), (0.003, 0.0)):
        P = one_surfel_scene([pos(2.0)], 0.2, math.log(o / (1 - o)))
        proj, img = render(P, cam)
        assert abs(img["alpha"][py, px] - expect) < 1e-12
    P = one_surfel_scene([pos(2.0)], 0.2, math.log(0.003 / 0.997))
    assert oracle.project(P, cam)["flags"][0] & oracle.F_OPACITY


def test_p4_invariants_tiny():
    w = scenes.workload(0)
    proj, off, ids, img = oracle.forward_view(w["scene"], w["cameras"][0])
    assert np.abs(img["alpha"] + img["T"] - 1).max() < 1e-15
    assert img["T"].min() >= 1e-4 and img["T"].max() <= 1
    has_med = img["med"] >= 0
    assert np.all(img["last"][has_med] > img["med"][has_med])
    assert img["n_con"] <= img["n_eval"]


def _brute_equal(sc, cam):
    proj = oracle.project(sc, cam)
    br = oracle.render_brute(proj, cam)
    rect = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    reach = oracle.bin_view(proj, cam)[:2]
    for off, ids in (rect, reach):  # the plain rect lists and the lists of the reach rule
        tl = oracle.render(proj, cam, off, ids)
        for k in ("rgb", "depth", "depth_med", "normal", "alpha", "T"):
            assert np.array_equal(tl[k], br[k]), k
        ids_ext = np.append(ids, -1)
        med_t = np.where(tl["med"] >= 0, ids_ext[np.where(tl["med"] >= 0, tl["med"], len(ids))], -1)
        assert np.array_equal(med_t, br["med_id"])


def test_p5_tiled_equals_brute_force_tiny():
    w = scenes.workload(0)
    _brute_equal(w["scene"], w["cameras"][0])


def test_p5_property_scenes():
    hyp = pytest.importorskip("hypothesis")
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=25, deadline=None, derandomize=True)
    @given(st.integers(1, 64), st.integers(0, 10_000), st.sampled_from([(16, 16), (33, 17), (48, 40)]),
           st.booleans())
    def run(n, seed, size, ties):
        rng = np.random.default_rng(seed)
        sc = scenes.tiny_scene(seed, n)
        sc.log_scale[:] = rng.uniform(np.log(0.01), np.log(0.6), size=sc.log_scale.shape).astype(np.float32)
        if ties:  # exact depth ties and edge-on surfels
            sc.mean[2] = np.round(sc.mean[2], 1)
            sc.quat[:, : n // 3] = np.array([[0.7071068], [0.7071068], [0.0], [0.0]], np.float32)
        sc.mean[:2] *= 1.6  # some centres off-screen
        _brute_equal(sc, scenes.tiny_camera(*size))

    run()


def test_p6_sort_matches_lexsort():
    w = scenes.workload(0)
    cam = w["cameras"][0]
    proj = oracle.project(w["scene"], cam)
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    tx = (cam.width + 15) // 16
    tiles, dbits, sid = [], [], []
    for i, r in enumerate(proj["tile_rect"]):
        for y in range(r[1], r[3]):
            for x in range(r[0], r[2]):
                tiles.append(y * tx + x)
                dbits.append(proj["depth32"][i:i + 1].view(np.uint32)[0])
                sid.append(i)
    order = np.lexsort((np.array(sid), np.array(dbits), np.array(tiles)))
    assert np.array_equal(np.array(sid)[order], ids)
    assert np.array_equal(np.bincount(np.array(tiles), minlength=len(off) - 1), np.diff(off))


def test_p7_bbox_contains_and_touches_conic():
    rng = np.random.default_rng(1)
    sc = scenes.tiny_scene(5, 200)
    cam = scenes.tiny_camera()
    proj = oracle.project(sc, cam)
    th = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
    checked = 0
    for i in rng.choice(200, 60, replace=False):
        if proj["flags"][i] & (oracle.F_CULLED):
            continue
        M = proj["M"][i].reshape(3, 3)
        k = math.sqrt(proj["k2"][i])
        pts = M @ np.stack([k * np.cos(th), k * np.sin(th), np.ones_like(th)])
        x, y = pts[0] / pts[2], pts[1] / pts[2]
        xlo, xhi, ylo, yhi = proj["bbox"][i]
        cx, cy = M[0, 2] / M[2, 2], M[1, 2] / M[2, 2]
        rf = k * math.sqrt(0.5)
        assert x.min() >= xlo - 1e-9 and x.max() <= xhi + 1e-9
        assert y.min() >= ylo - 1e-9 and y.max() <= yhi + 1e-9
        assert abs(min(x.min(), cx - rf) - xlo) < 1e-3 and abs(max(x.max(), cx + rf) - xhi) < 1e-3
        assert abs(min(y.min(), cy - rf) - ylo) < 1e-3 and abs(max(y.max(), cy + rf) - yhi) < 1e-3
        checked += 1
    assert checked > 20


def test_p8_sh_orthonormal_and_closed_forms():
    zs, wz = np.polynomial.legendre.leggauss(8)
    phis = np.arange(16) * 2 * np.pi / 16
    Z, PH = np.meshgrid(zs, phis, indexing="ij")
    WT = (wz[:, None] * np.full_like(PH, 2 * np.pi / 16)).ravel()
    r = np.sqrt(1 - Z ** 2)
    dirs = np.stack([r * np.cos(PH), r * np.sin(PH), Z], -1).reshape(-1, 3)
    Y, _ = oracle.sh_eval(3, dirs)
    G = (Y * WT[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12
    x, y, z = dirs.T
    pi = math.pi
    closed = {0: np.full_like(x, 0.5 / math.sqrt(pi)), 1: -math.sqrt(3 / (4 * pi)) * y,
              2: math.sqrt(3 / (4 * pi)) * z, 3: -math.sqrt(3 / (4 * pi)) * x,
              4: 0.5 * math.sqrt(15 / pi) * x * y, 6: 0.25 * math.sqrt(5 / pi) * (3 * z ** 2 - 1),
              8: 0.25 * math.sqrt(15 / pi) * (x ** 2 - y ** 2),
              12: 0.25 * math.sqrt(7 / pi) * z * (5 * z ** 2 - 3),
              15: -0.25 * math.sqrt(35 / (2 * pi)) * x * (x ** 2 - 3 * y ** 2)}
    for k, v in closed.items():
        assert np.abs(Y[:, k] - v).max() < 1e-12, k


def _fd_setup(seed=1, n=48, size=(32, 32)):
    rng = np.random.default_rng(seed)
    sc = scenes.tiny_scene(seed, n)
    sc.log_scale[:] += np.float32(1.0)
    cam = scenes.tiny_camera(*size)
    P = oracle._scene64(sc)
    H, W = cam.height, cam.width
    tgt = rng.uniform(size=(3, H, W))
    wts = dict(d_depth=rng.normal(size=(H, W)) * 1e-2, d_depth_med=rng.normal(size=(H, W)) * 1e-2,
               d_normal=rng.normal(size=(3, H, W)) * 1e-2, d_alpha=rng.normal(size=(H, W)) * 1e-2)

    def loss(P, M_override=None):
        proj = oracle.project(P, cam)
        if M_override is not None:
            proj["M"] = M_override
        off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], W, H)
        img = oracle.render(proj, cam, off, ids)
        lo = oracle.ssim_loss(img["rgb"], tgt)
        L = lo["loss"] + (wts["d_depth"] * img["depth"]).sum() + (wts["d_depth_med"] * img["depth_med"]).sum() \
            + (wts["d_normal"] * img["normal"]).sum() + (wts["d_alpha"] * img["alpha"]).sum()
        return L, img["sig"], (proj, off, ids, img, lo)

    return rng, cam, P, wts, loss


def test_p9_gradients_match_central_differences():
    rng, cam, P, wts, loss = _fd_setup()
    L0, sig0, (proj, off, ids, img, lo) = loss(P)
    up = dict(d_rgb=lo["d_total"], **wts)
    pg = oracle.backward_view(P, cam, proj, off, ids, up)["params"]
    eps = 1e-5
    checked = 0
    for name in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        flat = P[name].reshape(-1)
        fd, an = [], []
        for i in rng.choice(flat.size, size=min(25, flat.size), replace=False):
            Pp = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in P.items()}
            Pm = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in P.items()}
            Pp[name].reshape(-1)[i] += eps
            Pm[name].reshape(-1)[i] -= eps
            Lp, sp, _ = loss(Pp)
            Lm, sm, _ = loss(Pm)
            if not (np.array_equal(sp, sig0) and np.array_equal(sm, sig0)):
                continue  # a discrete decision changed inside +-eps
            fd.append((Lp - Lm) / (2 * eps))
            an.append(pg[name].reshape(-1)[i])
        fd, an = np.array(fd), np.array(an)
        assert len(fd) >= 10, name
        assert np.linalg.norm(fd - an) <= 1e-6 * np.linalg.norm(an) + 1e-12, name
        checked += len(fd)
    assert checked >= 80


def test_p10_viewspace_gradient_is_screen_translation_derivative():
    rng, cam, P, wts, loss = _fd_setup(seed=2, n=40)
    L0, sig0, (proj, off, ids, img, lo) = loss(P)
    g = oracle.backward_view(P, cam, proj, off, ids, dict(d_rgb=lo["d_total"], **wts), ndc=False)["g_total"]
    eps = 1e-5
    vis = np.where(proj["flags"] & F_VIS)[0]
    checked = 0
    for i in vis[:15]:
        for axis in (0, 1):
            res = []
            for sgn in (1, -1):
                M = proj["M"].copy().reshape(-1, 3, 3)
                M[i, axis, :] += sgn * eps * M[i, 2, :]
                L, s, _ = loss(P, M_override=M.reshape(-1, 9))
                res.append((L, s))
            if not (np.array_equal(res[0][1], sig0) and np.array_equal(res[1][1], sig0)):
                continue
            fd = (res[0][0] - res[1][0]) / (2 * eps)
            assert abs(fd - g[i, axis]) <= 1e-6 * max(abs(fd), 1e-6)
            checked += 1
    assert checked >= 10


def test_p11_dgd_hand_example_and_elongation():
    g_tot = np.array([[3.0, 4.0], [0.0, 1.0], [100.0, 100.0]])
    g_ssim = np.array([[1.0, 0.0], [0.0, 2.0], [50.0, 0.0]])
    vis = np.array([True, True, False])
    ls = np.log(np.array([[1.0, 1.0, 1.0], [1.0, 0.5, 0.01]]))
    st = oracle.new_densify_state(3)
    r = oracle.densify_stats(g_tot, g_ssim, vis, np.array([1.0, 2.0, 3.0]), ls, st, omega=0.9, eta_min=0.05,
                             grad_threshold=2.0)
    assert abs(r["scale"] - 1.8) < 1e-15               # max(0.9 * (5 + 1) / (1 + 2), 1)
    assert np.allclose(st["accum_dgd"], [1.8, 3.6, 0.0]) and np.allclose(st["accum_total"], [5.0, 1.0, 0.0])
    assert list(st["denom"]) == [1, 1, 0] and list(st["max_radius"]) == [1.0, 2.0, 0.0]
    assert np.allclose(r["eta"], [1.0, 0.5, 0.01])
    assert list(r["mask"] & 3) == [0, 1, 2]            # high: 3.6 >= 2; elongated: eta 0.01 < 0.05
    assert list(r["counters"][:6]) == [2, 1, 1, 0, 0, 1]
    # clamp at 1 when the SSIM gradients dominate
    st2 = oracle.new_densify_state(3)
    r2 = oracle.densify_stats(g_tot, g_ssim * 20, vis, np.ones(3), ls, st2)
    assert r2["scale"] == 1.0
    # the invisible surfel's gradients never enter the ratio
    g_tot2 = g_tot.copy()
    g_tot2[2] *= 1e6
    st3 = oracle.new_densify_state(3)
    assert oracle.densify_stats(g_tot2, g_ssim, vis, np.ones(3), ls, st3)["scale"] == r["scale"]
    # zero SSIM gradient -> factor 1
    st4 = oracle.new_densify_state(3)
    assert oracle.densify_stats(g_tot, g_ssim * 0, vis, np.ones(3), ls, st4)["scale"] == 1.0


def test_p12_ssim_identities_closed_form_and_fd():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(3, 20, 24))
    lo = oracle.ssim_loss(x, x)
    assert abs(lo["ssim"] - 1) < 1e-12 and abs(lo["loss"]) < 1e-12
    assert np.abs(lo["d_ssim"]).max() < 1e-12 and np.abs(lo["d_total"]).max() < 1e-12
    a, b = 0.3, 0.7
    lo = oracle.ssim_loss(np.full((3, 30, 30), a), np.full((3, 30, 30), b))
    C1 = 0.01 ** 2
    assert np.abs(lo["map"][:, 5:-5, 5:-5] - (2 * a * b + C1) / (a * a + b * b + C1)).max() < 1e-12
    x = rng.uniform(size=(3, 16, 16))
    y = rng.uniform(size=(3, 16, 16))
    lo = oracle.ssim_loss(x, y)
    # the L1 part is what separates the two gradients
    assert np.abs((lo["d_total"] - lo["d_ssim"]) - 0.8 * np.sign(x - y) / x.size).max() < 1e-15
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 7, 9), (2, 15, 3), (0, 8, 8), (1, 0, 15)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        lp, lm = oracle.ssim_loss(xp, y), oracle.ssim_loss(xm, y)
        assert abs((lp["loss"] - lm["loss"]) / (2 * eps) - lo["d_total"][idx]) < 1e-8
        s_fd = 0.2 * ((1 - lp["ssim"]) - (1 - lm["ssim"])) / (2 * eps)
        assert abs(s_fd - lo["d_ssim"][idx]) < 1e-8


# ---- P13 / P14: contribution-based trimming (Sec. 3.3, Eq. 3 and Eq. 4) ---------------------------

def _contrib(P, cam, gamma):
    proj = oracle.project(P, cam)
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    return proj, off, ids, oracle.contribution(proj, cam, off, ids, gamma)


def _facing_alpha(cam, z, scale, o):
    """alpha of a camera-facing isotropic surfel on the optical axis at depth z, per pixel sample."""
    i = np.arange(cam.width)[None, :] + 0.5
    j = np.arange(cam.height)[:, None] + 0.5
    X = (i - f32(cam.cx)) * z / f32(cam.fx)
    Y = (j - f32(cam.cy)) * z / f32(cam.fy)
    return np.minimum(0.99, o * np.exp(-(X ** 2 + Y ** 2) / (2 * scale ** 2)))


@pytest.mark.parametrize("gamma", [0.5, 0.25])
def test_p13_contribution_single_facing_surfel(gamma):
    cam = scenes.tiny_camera()
    logit = 1.3
    o = 1 / (1 + math.exp(-logit))
    P = one_surfel_scene([(0.0, 0.0, 0.0)], 0.3, logit)
    _, _, _, c = _contrib(P, cam, gamma)
    a = _facing_alpha(cam, 3.0, 0.3, o)
    region = a >= 1 / 255
    assert c["cnt"][0] == region.sum()
    # nothing lies in front: T = 1 at every pixel of the region
    assert abs(c["C"][0] - np.mean(a[region] ** gamma)) < 1e-12


def test_p13_contribution_two_stacked_surfels():
    cam = scenes.tiny_camera()
    gamma = 0.5
    o = 0.9
    logit = math.log(o / (1 - o))
    # front surfel at depth 2, back surfel at depth 2.5, both on the optical axis and facing the camera
    P = one_surfel_scene([(0.0, 0.0, -1.0), (0.0, 0.0, -0.5)], 0.3, logit)
    _, _, _, c = _contrib(P, cam, gamma)
    af = _facing_alpha(cam, 2.0, 0.3, o)
    ab = _facing_alpha(cam, 2.5, 0.3, o)
    front, back = af >= 1 / 255, ab >= 1 / 255
    T_back = np.where(front, 1 - af, 1.0)  # transmittance in front of the back surfel
    assert c["cnt"][0] == front.sum() and c["cnt"][1] == back.sum()
    assert abs(c["C"][0] - np.mean(af[front] ** gamma)) < 1e-12
    expect = np.mean(ab[back] ** gamma * T_back[back] ** (1 - gamma))
    assert abs(c["C"][1] - expect) < 1e-12


def test_p13_contribution_tiled_equals_brute_and_counts():
    w = scenes.workload(0)
    sc, cam = w["scene"], w["cameras"][0]
    proj = oracle.project(sc, cam)
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    for gamma in (0.5, 0.0, 1.0):
        t = oracle.contribution(proj, cam, off, ids, gamma)
        b = oracle.contribution_brute(proj, cam, gamma)
        assert np.array_equal(t["cnt"], b["cnt"])
        assert np.abs(t["sum"] - b["sum"]).max() <= 1e-12 * max(1.0, np.abs(b["sum"]).max())
    img = oracle.render(proj, cam, off, ids)
    assert t["cnt"].sum() == img["n_con"]
    # gamma = 0: the mean transmittance in front, within (0, 1]; gamma = 1: the mean alpha, within [1/255, 0.99]
    t0 = oracle.contribution(proj, cam, off, ids, 0.0)
    seen = t0["cnt"] > 0
    assert np.all(t0["C"][seen] <= 1) and np.all(t0["C"][seen] > 0)
    t1 = oracle.contribution(proj, cam, off, ids, 1.0)
    assert np.all(t1["C"][seen] >= 1 / 255 - 1e-15) and np.all(t1["C"][seen] <= 0.99 + 1e-15)
    assert np.all(t0["C"][~seen] == 0)


def test_p14_average_and_trim_bound():
    assert np.array_equal(oracle.average_contribution([[0, 1, 2], [2, 1, 0]]), [1.0, 1.0, 1.0])
    C = np.array([0.3, 0.0, 0.1, 0.0, 0.5, 0.2, 0.4, 0.1, 0.6, 0.05])
    # ratio .25 on 10 values: index floor(.25 * 9) = 2 of [0, 0, .05, .1, .1, .2, .3, .4, .5, .6]
    bound, mask = oracle.trim_threshold(C, 0.25)
    assert bound == 0.05 and list(np.flatnonzero(mask)) == [1, 3, 9]
    bound, mask = oracle.trim_threshold(C, 0.1)   # index 0: the never-seen surfels only
    assert bound == 0.0 and list(np.flatnonzero(mask)) == [1, 3]
    bound, mask = oracle.trim_threshold(C, 0.4)   # index 3; ties at the bound are removed too
    assert bound == 0.1 and list(np.flatnonzero(mask)) == [1, 2, 3, 7, 9]
    bound, mask = oracle.trim_threshold(C, 1.0)
    assert bound == 0.6 and mask.all()


# ---- P15: densification action ---------------------------------------------------------------------

def test_p15_densify_actions_and_apply_by_hand():
    n = 6
    mean = np.array([[0.0, 1.0, 2.0, 3.0, 4.0, 5.0],
                     [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                     [1.0, 1.0, 1.0, 1.0, 1.0, 1.0]])
    su = np.array([0.01, 0.01, 0.2, 0.2, 0.01, 0.3])
    sv = np.array([0.01, 0.005, 0.1, 0.2, 0.01, 0.1])
    log_scale = np.log(np.stack([su, sv]))
    c45 = math.cos(math.pi / 4)
    quat = np.array([[1, 1, 1, 1, 1, c45], [0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, c45]], np.float64)
    logit = np.array([2.0, 2.0, 2.0, 2.0, -6.0, 2.0])   # surfel 4: opacity 0.0025
    sh = np.arange(16 * 3 * n, dtype=np.float64).reshape(16, 3, n)
    P = dict(mean=mean, log_scale=log_scale, quat=quat, opacity_logit=logit, sh=sh, sh_degree=3)
    cand = np.array([0, 1, 1, 1, 1, 1], bool)
    remove = np.array([0, 0, 0, 1, 0, 0], bool)
    act = oracle.densify_actions(cand, remove, log_scale, logit, dense_scale=0.05, min_opacity=0.005)
    assert list(act) == [0, 1, 2, 3, 3, 2]
    z = np.zeros((n, 2, 2))
    z[2] = [[1.0, -2.0], [0.5, 0.25]]
    z[5] = [[1.0, 0.0], [0.0, 1.0]]
    out = oracle.densify_apply(P, act, z)
    # survivors 0, 1; then the copy of 1, the children of 2, the children of 5
    src = [0, 1, 1, 2, 2, 5, 5]
    assert out["mean"].shape == (3, 7) and out["sh"].shape == (16, 3, 7)
    assert np.array_equal(out["sh"], sh[:, :, src])
    assert np.array_equal(out["quat"], quat[:, src]) and np.array_equal(out["opacity_logit"], logit[src])
    # identity rotation: children at mu + (s_u z0, s_v z1, 0), scales / 1.6
    assert np.allclose(out["mean"][:, 3], [2 + 0.2 * 1.0, 0.1 * -2.0, 1.0], atol=1e-15)
    assert np.allclose(out["mean"][:, 4], [2 + 0.2 * 0.5, 0.1 * 0.25, 1.0], atol=1e-15)
    assert np.allclose(out["log_scale"][:, 3], np.log([0.2 / 1.6, 0.1 / 1.6]), atol=1e-15)
    # a quarter turn about the normal maps the tangent u onto +y and v onto -x
    assert np.allclose(out["mean"][:, 5], [5.0, 0.3, 1.0], atol=1e-15)
    assert np.allclose(out["mean"][:, 6], [5.0 - 0.1, 0.0, 1.0], atol=1e-15)
    # survivors and clones are unchanged copies
    assert np.array_equal(out["mean"][:, :3], mean[:, [0, 1, 1]])
    assert np.array_equal(out["log_scale"][:, :3], log_scale[:, [0, 1, 1]])
    keep, clone, split = (act == 0).sum(), (act == 1).sum(), (act == 2).sum()
    assert out["mean"].shape[1] == keep + 2 * clone + 2 * split


def test_p15_slots_follow_the_apply_order():
    rng = np.random.default_rng(15)
    n = 40
    act = rng.integers(0, 4, n).astype(np.int32)
    dst, src, kind = oracle.densify_slots(act)
    # the apply with ids planted in the opacity field and z = 0 reproduces the slot order
    P = dict(mean=np.zeros((3, n)), log_scale=np.zeros((2, n)), quat=np.tile([[1.0], [0], [0], [0]], (1, n)),
             opacity_logit=np.arange(n, dtype=np.float64), sh=np.zeros((1, 3, n)), sh_degree=0)
    out = oracle.densify_apply(P, act, np.zeros((n, 2, 2)))
    assert np.array_equal(out["opacity_logit"], src.astype(np.float64))
    assert len(src) == (act == 0).sum() + 2 * (act == 1).sum() + 2 * (act == 2).sum()
    for i in range(n):
        assert (dst[0, i] >= 0) == (act[i] in (0, 1)) and (dst[1, i] >= 0) == (act[i] in (1, 2))
        if dst[0, i] >= 0:
            assert src[dst[0, i]] == i and kind[dst[0, i]] == 0
        if act[i] == 1:
            assert src[dst[1, i]] == i and kind[dst[1, i]] == 1
        if act[i] == 2:
            assert list(src[dst[1, i]:dst[1, i] + 2]) == [i, i] and list(kind[dst[1, i]:dst[1, i] + 2]) == [2, 3]
    # survivors first, new surfels after, each group in id order
    surv = (act == 0) | (act == 1)
    assert np.all(np.diff(src[:surv.sum()]) > 0) and np.all(np.diff(src[surv.sum():]) >= 0)


# ---- P16: visibility frequency for the crop volume --------------------------------------------------

def _cam100(R=None, t=None, W=100, H=100, f=100.0):
    return scenes.Camera(W, H, f, f, W / 2.0, H / 2.0, np.eye(3) if R is None else np.asarray(R, np.float64),
                         np.zeros(3) if t is None else np.asarray(t, np.float64))


def test_p16_sphere_box_closed_form_on_axis():
    from oracle import visibility as vis
    for Z, rho in ((10.0, 1.0), (3.0, 2.5), (100.0, 0.01)):
        u0, u1, v0, v1 = vis.sphere_image_bbox(np.array(0.0), np.array(0.0), np.array(Z), rho, 100.0, 80.0, 50.0, 40.0)
        half = rho / math.sqrt(Z * Z - rho * rho)   # tan of the half-angle asin(rho / Z)
        assert np.isclose(u0, 50.0 - 100.0 * half, rtol=0, atol=1e-12)
        assert np.isclose(u1, 50.0 + 100.0 * half, rtol=0, atol=1e-12)
        assert np.isclose(v0, 40.0 - 80.0 * half, rtol=0, atol=1e-12)
        assert np.isclose(v1, 40.0 + 80.0 * half, rtol=0, atol=1e-12)


def test_p16_sphere_box_against_silhouette_sampling():
    from oracle import visibility as vis
    rng = np.random.default_rng(16)
    # dense sphere surface samples: the projected samples fill the image, whose box is the exact box
    k = 400
    th, ph = np.meshgrid(np.linspace(0, np.pi, k), np.linspace(0, 2 * np.pi, 2 * k), indexing="ij")
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 0).reshape(3, -1)
    for _ in range(20):
        X, Y = rng.uniform(-20, 20, 2)
        Z = rng.uniform(2, 40)
        rho = rng.uniform(0.05, 0.9) * min(Z, 2.0)
        pts = np.array([[X], [Y], [Z]]) + rho * S
        u = 120.0 * pts[0] / pts[2] + 64.0
        v = 90.0 * pts[1] / pts[2] + 48.0
        u0, u1, v0, v1 = vis.sphere_image_bbox(X, Y, Z, rho, 120.0, 90.0, 64.0, 48.0)
        scale = max(1.0, abs(u0), abs(u1), abs(v0), abs(v1))
        assert u.min() >= u0 - 1e-9 * scale and u.max() <= u1 + 1e-9 * scale
        assert v.min() >= v0 - 1e-9 * scale and v.max() <= v1 + 1e-9 * scale
        # the box is touched: sampling resolution ~ (pi / k)^2 / 2 of the extent
        tol = 2e-4 * (u1 - u0) + 1e-9
        assert u.min() - u0 < tol and u1 - u.max() < tol
        assert v.min() - v0 < 2e-4 * (v1 - v0) + 1e-9 and v1 - v.max() < 2e-4 * (v1 - v0) + 1e-9


def test_p16_visible_mask_by_hand():
    from oracle import visibility as vis
    cam = _cam100()
    # image centre (u = 50 lies between the samples 49.5 and 50.5: a 0.7 px reach covers both, 0.3 px
    # none); behind the camera; closer than znear
    P = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [10.0, -10.0, 0.1]])
    v, f = vis.visible(P, cam, 0.01, 0.7)
    assert list(v) == [True, False, False] and not f.any()
    assert list(vis.visible(P, cam, 0.01, 0.3)[0]) == [False, False, False]
    # a tiny footprint between the samples x = 59.5 and 60.5 (centre u = 60.0, reach 0.3 px): hidden;
    # moved to u = 60.3 it covers 60.5: visible.  (Z = 10, f = 100: X = (u - 50) / 10; v = 50.5 sits
    # on a sample row.)
    P = np.array([[1.0, 1.03], [0.05, 0.05], [10.0, 10.0]])
    v, f = vis.visible(P, cam, 1e-4, 0.3)
    assert list(v) == [False, True] and not f.any()
    # centre 3 px left of the image (u = -3): a reach of 3.6 px covers the sample 0.5 of column 0, 3.2 px
    # does not (rho = 0 leaves only the filter disc)
    P = np.array([[-5.3], [0.0], [10.0]])
    assert list(vis.visible(P, cam, 0.0, 3.6)[0]) == [True]
    assert list(vis.visible(P, cam, 0.0, 3.2)[0]) == [False]
    # a sphere reaching the camera plane is visible whatever its image
    P = np.array([[30.0], [0.0], [0.5]])
    assert list(vis.visible(P, cam, 1.0, 0.3)[0]) == [True]


def test_p16_counts_are_sums_over_views_and_crop():
    from oracle import visibility as vis
    rng = np.random.default_rng(160)
    P = rng.uniform(-5, 5, (3, 500))
    P[2] += 20.0
    cams = [_cam100(t=[rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-5, 5)]) for _ in range(7)]
    cnt, frag = vis.visibility_count(P, cams, 0.05, 0.7)
    assert np.array_equal(cnt, sum(vis.visible(P, c, 0.05, 0.7)[0].astype(np.int64) for c in cams))
    assert cnt.min() >= 0 and cnt.max() <= 7 and frag.sum() == 0
    tau = 4
    keep, G, h0, h1 = vis.crop_volume(P, cnt, tau, np.hstack([np.eye(3), np.zeros((3, 1))]))
    P32 = P.astype(np.float32).astype(np.float64)
    assert np.array_equal(keep, cnt >= tau)
    assert np.array_equal(G, P32[:2, keep]) and h0 == P32[2, keep].min() and h1 == P32[2, keep].max()
    # a transform that makes y the height axis and shifts it
    T = np.array([[1.0, 0, 0, 0], [0, 0, 1.0, 0], [0, 1.0, 0, -2.0]])
    keep, G, h0, h1 = vis.crop_volume(P, cnt, tau, T)
    assert np.array_equal(G, np.stack([P32[0, keep], P32[2, keep]])) and h0 == P32[1, keep].min() - 2.0
    keep, G, h0, h1 = vis.crop_volume(P, cnt, 8, T)
    assert not keep.any() and G.shape == (2, 0) and math.isnan(h0)


# ---- P17: serving storage (float16 + vector quantization) ------------------------------------------

def test_p17_float16_and_partition():
    from oracle import compact as oc
    # IEEE half: 1/3 -> 0x3555, the largest finite 65504, 2049 rounds to the even 2048, 2051 to 2052
    v = np.array([1 / 3, 65504.0, 2049.0, 2051.0, -0.0], np.float32).astype(np.float16)
    assert list(v.view(np.uint16)) == [0x3555, 0x7BFF, 0x6800, 0x6802, 0x8000]
    order, nf = oc.order_partition(np.array([1, 0, 0, 1, 0, 1], np.uint8))
    assert list(order) == [1, 2, 4, 0, 3, 5] and nf == 3


def test_p17_nearest_codeword():
    from oracle import compact as oc
    rng = np.random.default_rng(17)
    C = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0], [10.0, 10.0]])
    X = C[[3, 0, 2, 1, 1]] + rng.uniform(-1, 1, (5, 2))
    codes, best, gap = oc.vq_assign(X, C)
    assert list(codes) == [3, 0, 2, 1, 1] and np.all(gap > 0.1)
    # equal distances: the smaller index
    codes, _, gap = oc.vq_assign(np.array([[5.0, 0.0]]), C)
    assert codes[0] == 0 and gap[0] == 0.0
    # against explicit loops
    X = rng.normal(size=(50, 6))
    C = rng.normal(size=(9, 6))
    codes, best, _ = oc.vq_assign(X, C)
    for i in range(50):
        d = [sum((X[i, k] - C[j, k]) ** 2 for k in range(6)) for j in range(9)]
        assert codes[i] == int(np.argmin(d)) and math.isclose(best[i], min(d), rel_tol=1e-12)


def test_p17_lloyd_update_and_monotone_error():
    from oracle import compact as oc
    X = np.array([[0.0, 0.0], [2.0, 0.0], [10.0, 10.0], [12.0, 10.0], [11.0, 13.0]])
    C0 = np.array([[1.0, 1.0], [10.0, 10.0], [50.0, 50.0]])
    codes, _, _ = oc.vq_assign(X, C0)
    assert list(codes) == [0, 0, 1, 1, 1]
    C1, cnt = oc.vq_update(X, codes, C0)
    assert np.allclose(C1, [[1.0, 0.0], [11.0, 11.0], [50.0, 50.0]]) and list(cnt) == [2, 3, 0]
    rng = np.random.default_rng(170)
    Y = np.concatenate([rng.normal(c, 0.3, (200, 3)) for c in rng.uniform(-5, 5, (12, 3))])
    _, _, errs = oc.kmeans(Y, 12, 8)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))


def test_p17_decode_of_pack_within_half_rounding():
    from oracle import compact as oc
    sc = scenes.tiny_scene(17, 600, sh_degree=2)
    P = dict(mean=sc.mean, log_scale=sc.log_scale, quat=sc.quat, opacity_logit=sc.opacity_logit, sh=sc.sh,
             sh_degree=2)
    q = (np.arange(600) % 3 == 0).astype(np.uint8)
    order, nf = oc.order_partition(q)
    X = sc.sh[:, :, order[nf:]].transpose(2, 0, 1).reshape(600 - nf, 27)
    C, codes, _ = oc.kmeans(X, 16, 3)
    c = oc.pack(P, order, nf, codes, C)
    d = oc.decode(c)
    assert np.array_equal(d["mean"], sc.mean[:, order])
    for k in ("log_scale", "quat"):
        ref = np.asarray(P[k], np.float64)[:, order]
        assert np.all(np.abs(d[k] - ref) <= 2.0 ** -11 * np.abs(ref) + 2.0 ** -24)
    ref = sc.sh[:, :, order[:nf]].astype(np.float64)
    assert np.all(np.abs(d["sh"][:, :, :nf] - ref) <= 2.0 ** -11 * np.abs(ref) + 2.0 ** -24)
    # a quantized surfel decodes to its float16 codeword
    cw = C[codes[0]].astype(np.float32).astype(np.float16).astype(np.float32).reshape(9, 3)
    assert np.array_equal(d["sh"][:, :, nf], cw)


# ---- P18 the list rule ------------------------------------------------------------------------------

def _pixel_rho(M, x, y):
    """rho = min(rho3d, rho2d) of surfels M [m][9] at pixel samples x, y [m][k] (written out from Eq. 1's
    ray-splat intersection: p = (x m3 - m1) x (y m3 - m2), u = p0 / p2, v = p1 / p2)."""
    m1, m2, m3 = M[:, None, 0:3], M[:, None, 3:6], M[:, None, 6:9]
    a = x[..., None] * m3 - m1
    b = y[..., None] * m3 - m2
    p = np.cross(a, b)
    with np.errstate(divide="ignore", invalid="ignore"):
        rho3 = np.where(p[..., 2] != 0, (p[..., 0] ** 2 + p[..., 1] ** 2) / p[..., 2] ** 2, np.inf)
    cx, cy = M[:, 2] / M[:, 8], M[:, 5] / M[:, 8]
    rho2 = 2 * ((x - cx[:, None]) ** 2 + (y - cy[:, None]) ** 2)
    return np.minimum(rho3, rho2)


def test_p18_facing_surfel_keeps_tiles_within_its_radius():
    cam = scenes.tiny_camera(256, 256)
    for scale, logit in ((0.3, 1.3), (0.12, -1.0), (0.004, 2.0)):
        P = one_surfel_scene([(0.05, -0.03, 0.0)], scale, logit)
        proj = oracle.project(P, cam)
        keep, fragile = oracle.tile_reach(proj)
        sid, tile = oracle.rect_tiles(proj["tile_rect"], cam.width)
        o = 1 / (1 + math.exp(-logit))
        K = 2 * math.log(255 * o) * (1 + 2e-3) + 2e-3
        # camera at distance 3 on the axis: plane units = screen offsets * 3 / f
        R = max(math.sqrt(K) * scale * f32(cam.fx) / 3.0, math.sqrt(K / 2))
        M = proj["M"][0]
        cx, cy = M[2] / M[8], M[5] / M[8]
        tx = (cam.width + 15) // 16
        x0, y0 = 16.0 * (tile % tx), 16.0 * (tile // tx)
        pad = 1 / 64
        dx = np.maximum(np.maximum(x0 + 0.5 - pad - cx, cx - (x0 + 15.5 + pad)), 0)
        dy = np.maximum(np.maximum(y0 + 0.5 - pad - cy, cy - (y0 + 15.5 + pad)), 0)
        expect = dx * dx + dy * dy <= R * R
        assert not fragile.any() or fragile.sum() <= 2
        assert np.array_equal(keep[~fragile], expect[~fragile]), scale
        if scale == 0.3:
            assert (~keep).sum() >= 4  # the rect's corner tiles lie outside the circle


def _elongated_scene(seed, n):
    rng = np.random.default_rng(seed)
    sc = scenes.tiny_scene(seed, n)
    su = rng.uniform(np.log(0.02), np.log(0.3), n)
    ratio = np.log(rng.uniform(5, 50, n))
    sc.log_scale[0] = (su + ratio / 2).astype(np.float32)
    sc.log_scale[1] = (su - ratio / 2).astype(np.float32)
    sc.mean[:2] *= 1.4
    return sc


@pytest.mark.parametrize("seed", [3, 4])
def test_p18_no_reachable_tile_dropped_brute_force(seed):
    sc = _elongated_scene(seed, 300)
    cam = scenes.tiny_camera(160, 112)
    proj = oracle.project(sc, cam)
    keep, fragile = oracle.tile_reach(proj)
    sid, tile = oracle.rect_tiles(proj["tile_rect"], cam.width)
    tx = (cam.width + 15) // 16
    lx, ly = np.meshgrid(np.arange(16) + 0.5, np.arange(16) + 0.5)
    x = (16 * (tile % tx))[:, None] + lx.reshape(-1)[None, :]
    y = (16 * (tile // tx))[:, None] + ly.reshape(-1)[None, :]
    rho = _pixel_rho(proj["M"][sid], x, y)
    inside = (rho <= proj["k2"][sid][:, None]).any(1)
    assert inside.sum() > 200
    assert not np.any(inside & ~keep), "a tile with a pixel sample inside the cutoff region was dropped"
    # tight: what is kept but holds no sample inside the region is a small share of the rect's dropouts
    assert (~keep).sum() > 0.3 * (~inside).sum()
    assert fragile.sum() <= max(2, int(1e-3 * keep.size))
    _brute_equal(sc, cam)
