"""More pins of the FP64 oracle to the mathematics (no GPU): the surfel geometry, the SH view direction
and the FP32 error model behind the decision margins.

P19 the 2DGS surfel (Sec. 3.1): the tangents t_u, t_v and the normal are the columns of the rotation of
    the quaternion, checked against scipy's rotation on random surfels and cameras; a camera-facing
    surfel with s_u = 3 s_v turned about its normal by a quarter and by a twelfth of a turn has, at every
    pixel sample, the alpha of the hand-derived ellipse (elongated along screen y for the quarter turn,
    mirrored if the tangents were taken from the rotation's rows); a surfel tilted 60 and 120 degrees
    about x has the alpha, the intersection depth and the normal of the closed-form ray-plane
    intersection, flipped towards the camera only when it faces away
P20 the SH view direction (Sec. 3.1 colour): with a single degree-1 or degree-3 coefficient the colour is
    0.5 + f Y(d) at d = (mu - C) / |mu - C| with C = -R^T t the camera centre (odd degrees change sign
    with d), under a rotated camera, at SH degrees 1 to 3; a negative sum clamps to 0
P21 the FP32 error model: an emulated FP32 evaluation (coefficients of the ray-splat map and the pixel
    offsets rounded to float32, float32 arithmetic) of sampled (pixel, surfel) pairs of an aerial view
    with 10 % degenerate surfels (axis ratio 50-1000) stays within the model's bounds of rho, alpha and
    the transmittance (the bounds carry a safety factor of 3; the emulated error must stay below 1.5x
    the bound without it)
"""
import math

import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes

F32 = lambda v: float(np.float32(v))


def _surfels(mu, log_scale, quat, logit=2.0, deg=3, sh=None):
    mu = np.asarray(mu, np.float64).reshape(-1, 3)
    n = mu.shape[0]
    K = (deg + 1) ** 2
    s = np.zeros((K, 3, n)) if sh is None else np.asarray(sh, np.float64)
    if sh is None:
        s[0] = 1.0
    return dict(mean=mu.T.copy(), log_scale=np.asarray(log_scale, np.float64).reshape(2, n),
                quat=np.asarray(quat, np.float64).reshape(4, n), opacity_logit=np.full(n, float(logit)), sh=s,
                sh_degree=deg)


def _render(P, cam):
    proj = oracle.project(P, cam)
    off, ids = oracle.bin_tiles(proj["tile_rect"], proj["depth32"], cam.width, cam.height)
    return proj, oracle.render(proj, cam, off, ids)


def _samples(cam):
    i = np.arange(cam.width)[None, :] + 0.5
    j = np.arange(cam.height)[:, None] + 0.5
    return i, j


def _alpha(o, rho):
    a = np.minimum(0.99, o * np.exp(-0.5 * rho))
    return np.where(a < 1 / 255, 0.0, a)


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


# ---------------------------------------------------------------------------------------------------
# P19 geometry
# ---------------------------------------------------------------------------------------------------

def test_p19_screen_transform_from_library_rotation():
    """M = K [R_c s_u t_u | R_c s_v t_v | R_c mu + t] with (t_u, t_v, n) the columns of scipy's rotation
    of the quaternion, and the camera-space normal = +-R_c n facing the camera (n . (R_c mu + t) <= 0)."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(19)
    n = 64
    q = rng.normal(size=(4, n))
    mu = rng.uniform(-1, 1, (n, 3))
    ls = rng.uniform(math.log(0.02), math.log(0.3), (2, n))
    P = _surfels(mu, ls, q)
    for k in range(3):
        cam = scenes.tiny_camera(96, 80)
        cam.R = _rot_y(0.4 * k - 0.3) @ _rot_x(0.2 * k - 0.1)
        cam.t = np.array([0.1 * k, -0.2, 3.0 + 0.3 * k])
        proj = oracle.project(P, cam)
        a = cam.as_array()
        fx, fy, cx, cy = a[2:6]
        Rc, t = a[6:15].reshape(3, 3), a[15:18]
        Kmat = np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1]])
        Rw = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], 1)).as_matrix()  # scipy takes (x, y, z, w)
        s = np.exp(ls)
        for i in range(n):
            cols = np.stack([Rc @ (s[0, i] * Rw[i][:, 0]), Rc @ (s[1, i] * Rw[i][:, 1]), Rc @ mu[i] + t], 1)
            Mref = Kmat @ cols
            assert np.abs(proj["M"][i] - Mref.ravel()).max() <= 1e-12 * max(1.0, np.abs(Mref).max())
            nc = Rc @ Rw[i][:, 2]
            pc = Rc @ mu[i] + t
            sgn = -1.0 if nc @ pc > 0 else 1.0
            assert np.abs(proj["normal"][i] - sgn * nc).max() <= 1e-12
            assert proj["normal"][i] @ pc <= 0


@pytest.mark.parametrize("phi_deg", [90.0, 30.0])
def test_p19_facing_anisotropic_surfel_turned_about_its_normal(phi_deg):
    """s_u = 3 s_v, turned by phi about the normal (quaternion (cos phi/2, 0, 0, sin phi/2)) at the origin,
    facing the camera at distance 3: the ray through (x, y) meets the plane at (X, Y) = ((x - cx) 3 / fx,
    (y - cy) 3 / fy), u = (X cos phi + Y sin phi) / s_u, v = (-X sin phi + Y cos phi) / s_v."""
    cam = scenes.tiny_camera()
    su, sv = 0.3, 0.1
    phi = math.radians(phi_deg)
    logit = 1.7
    o = 1 / (1 + math.exp(-logit))
    P = _surfels([(0, 0, 0)], [math.log(su), math.log(sv)], [math.cos(phi / 2), 0, 0, math.sin(phi / 2)], logit)
    proj, img = _render(P, cam)
    i, j = _samples(cam)
    X = (i - F32(cam.cx)) * 3.0 / F32(cam.fx)
    Y = (j - F32(cam.cy)) * 3.0 / F32(cam.fy)
    u = (X * math.cos(phi) + Y * math.sin(phi)) / su
    v = (-X * math.sin(phi) + Y * math.cos(phi)) / sv
    rho3 = u * u + v * v
    rho2 = 2 * ((i - F32(cam.cx)) ** 2 + (j - F32(cam.cy)) ** 2)
    a = _alpha(o, np.minimum(rho3, rho2))
    assert (a > 0).sum() > 200
    assert np.abs(img["alpha"] - a).max() < 1e-12
    assert np.abs(img["depth"] - 3 * a).max() < 1e-12
    assert np.abs(img["normal"][2] + a).max() < 1e-12
    ys, xs = np.nonzero(img["alpha"] > 0)
    if phi_deg == 90.0:  # the long axis t_u = (0, 1, 0) lies along screen y
        assert ys.max() - ys.min() > 2.5 * (xs.max() - xs.min())
    else:  # long axis along (cos 30, sin 30): x and y of the covered pixels correlate positively (y down)
        assert np.corrcoef(xs, ys)[0, 1] > 0.5


@pytest.mark.parametrize("theta_deg", [60.0, 120.0])
def test_p19_tilted_surfel_alpha_depth_normal(theta_deg):
    """A surfel at the origin turned by theta about x: t_u = (1, 0, 0), t_v = (0, cos, sin), n = (0, -sin,
    cos).  The camera ray C + lam d, C = (0, 0, -3), d = ((x - cx) / fx, (y - cy) / fy, 1), meets the plane
    n . X = 0 at lam = 3 cos / (cos - sin d_y): the intersection depth is lam, (u, v) = (lam d_x / s_u,
    (cos lam d_y + sin (lam - 3)) / s_v).  The normal faces the camera: flipped when n . (0, 0, 3) > 0."""
    cam = scenes.tiny_camera()
    th = math.radians(theta_deg)
    c, s = math.cos(th), math.sin(th)
    su, sv = 0.25, 0.15
    logit = 2.2
    o = 1 / (1 + math.exp(-logit))
    P = _surfels([(0, 0, 0)], [math.log(su), math.log(sv)], [math.cos(th / 2), math.sin(th / 2), 0, 0], logit)
    proj, img = _render(P, cam)
    i, j = _samples(cam)
    fx, fy, cx, cy = F32(cam.fx), F32(cam.fy), F32(cam.cx), F32(cam.cy)
    dx, dy = (i - cx) / fx, (j - cy) / fy
    den = c - s * dy
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = np.where(np.abs(den) > 0, 3 * c / den, np.inf)
        front = lam > 0
        u = lam * dx / su
        v = (c * lam * dy + s * (lam - 3)) / sv
        rho3 = np.where(front, u * u + v * v, np.inf)
    rho2 = 2 * ((i - cx) ** 2 + (j - cy) ** 2)
    is3d = rho3 <= rho2
    a = _alpha(o, np.where(is3d, rho3, rho2))
    zf = np.where(is3d, lam, 3.0)
    assert (a > 0).sum() > 200
    assert np.abs(img["alpha"] - a).max() < 1e-12
    on = a > 0
    assert np.abs(img["depth"] - np.where(on, a * zf, 0)).max() < 1e-9
    assert np.abs(img["depth_med"] - np.where(on, zf, 0)).max() < 1e-9
    # the depth varies along the centre column (it is a tilted plane) and not along the centre row
    col = np.where(on[:, 64], img["depth_med"][:, 64], np.nan)
    assert np.nanmax(col) - np.nanmin(col) > 0.05
    n_face = np.array([0.0, -s, c]) * (-1.0 if 3 * c > 0 else 1.0)
    for k in range(3):
        assert np.abs(img["normal"][k] - a * n_face[k]).max() < 1e-12
    assert np.allclose(proj["normal"][0], n_face, atol=1e-15)


# ---------------------------------------------------------------------------------------------------
# P20 SH view direction
# ---------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("deg", [1, 2, 3])
def test_p20_sh_view_direction(deg):
    """colour = max(0, 0.5 + sum f Y(d)) at d = (mu - C) / |mu - C|, C = -R^T t.  Red carries Y_1^0
    (= sqrt(3/4pi) z), green Y_1^1 (= -sqrt(3/4pi) x), blue Y_1^-1 (= -sqrt(3/4pi) y); at degree 3 red also
    carries Y_3^0 (= sqrt(7/pi) / 4 z (5 z^2 - 3)), at degree 2 blue carries Y_2^-2 (= sqrt(15/pi) / 2 x y)."""
    rng = np.random.default_rng(20 + deg)
    n = 12
    mu = rng.uniform(-1, 1, (n, 3))
    K = (deg + 1) ** 2
    sh = np.zeros((K, 3, n))
    f = rng.uniform(-0.8, 0.8, (5, n))
    sh[2, 0], sh[3, 1], sh[1, 2] = f[0], f[1], f[2]
    if deg >= 3:
        sh[12, 0] = f[3]
    if deg >= 2:
        sh[4, 2] = f[4]
    P = _surfels(mu, np.full((2, n), math.log(0.1)), np.tile([[1.0], [0], [0], [0]], (1, n)), 1.0, deg, sh)
    cam = scenes.tiny_camera()
    cam.R = _rot_y(0.5) @ _rot_x(-0.3)
    Cw = np.array([-1.2, 0.8, -2.6])
    cam.t = -cam.R @ Cw
    proj = oracle.project(P, cam)
    a = cam.as_array()
    Rc, t = a[6:15].reshape(3, 3), a[15:18]
    C = -Rc.T @ t
    d = mu - C
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x, y, z = d.T
    k1 = math.sqrt(3 / (4 * math.pi))
    red = 0.5 + f[0] * k1 * z + (f[3] * math.sqrt(7 / math.pi) / 4 * z * (5 * z * z - 3) if deg >= 3 else 0)
    green = 0.5 - f[1] * k1 * x
    blue = 0.5 - f[2] * k1 * y + (f[4] * math.sqrt(15 / math.pi) / 2 * x * y if deg >= 2 else 0)
    ref = np.stack([red, green, blue], 1)
    assert np.abs(proj["rgb_raw"] - ref).max() < 1e-13
    assert np.abs(proj["rgb"] - np.maximum(ref, 0)).max() < 1e-13
    # the reversed direction changes every odd term: it would miss by far more than the tolerance
    red_rev = 0.5 - f[0] * k1 * z
    assert np.abs(proj["rgb_raw"][:, 0] - red_rev).max() > 1e-3


def test_p20_negative_colour_clamps_to_zero():
    P = _surfels([(0.0, 0.0, 0.0)], [[math.log(0.1)], [math.log(0.1)]], [1.0, 0, 0, 0], 1.0, 0,
                 np.array([[[-3.0], [0.2], [0.0]]]))
    proj = oracle.project(P, scenes.tiny_camera())
    y00 = 0.5 / math.sqrt(math.pi)
    assert abs(proj["rgb_raw"][0, 0] - (0.5 - 3.0 * y00)) < 1e-15 and proj["rgb"][0, 0] == 0.0
    assert abs(proj["rgb"][0, 1] - (0.5 + 0.2 * y00)) < 1e-15 and abs(proj["rgb"][0, 2] - 0.5) < 1e-15


# ---------------------------------------------------------------------------------------------------
# P21 the FP32 error model of the decision margins
# ---------------------------------------------------------------------------------------------------

SAFETY = 3.0   # the model's safety factor (its bounds are SAFETY x the first-order estimate)
SLACK = 1.5    # emulated error / (bound / SAFETY) must stay below this


def _degenerate_view(seed=21):
    """A miniature of the 10 M-surfel aerial workload: the same surfel spacing (0.32 m), log-normal scales
    (sigma 0.6) and 10 % degenerate surfels (axis ratio 50-1000), and the same pixel footprint (a 320 px
    wide view from 20-60 m instead of 1600 px from 100-300 m)."""
    city = scenes.make_city(seed, L=100.0, n_boxes=2)
    city.boxes[:, 4] = 4.0  # low sheds: the cameras fly 20-60 m above the ground
    sc = scenes.city_scene(seed, 100_000, L=100.0, city=city, elongated_frac=0.10, elong_range=(50.0, 1000.0),
                           lognormal_sigma=0.6)
    cam = scenes.aerial_cameras(seed + 1000, city, count=1, width=320, height=213, alt=(20.0, 60.0))[0]
    return sc, cam


def _f32_map(M):
    """Coefficients of p(x', y') = x' px + y' py + p0 about the projected centre (FP64) and the centre."""
    M = M.reshape(-1, 3, 3)
    m1, m2, m3 = M[:, 0], M[:, 1], M[:, 2]
    cx, cy = M[:, 0, 2] / M[:, 2, 2], M[:, 1, 2] / M[:, 2, 2]
    a0 = cx[:, None] * m3 - m1
    b0 = cy[:, None] * m3 - m2
    return np.cross(m3, b0), np.cross(a0, m3), np.cross(a0, b0), cx, cy


def _emulate(M, o, x, y):
    """FP32 evaluation: map coefficients rounded to float32, the pixel offset taken relative to the
    16-px tile origin (centre offset rounded once), then float32 arithmetic for p, u, v, rho3, rho2 and
    alpha = exp2(log2 o - rho log2(e) / 2)."""
    f = np.float32
    px, py, p0, cx, cy = _f32_map(M)
    x0, y0 = np.floor(x / 16) * 16, np.floor(y / 16) * 16
    dx = (x - x0).astype(f) - (cx - x0).astype(f)
    dy = (y - y0).astype(f) - (cy - y0).astype(f)
    p = dx[:, None] * px.astype(f) + dy[:, None] * py.astype(f) + p0.astype(f)
    u, v = p[:, 0] / p[:, 2], p[:, 1] / p[:, 2]
    rho3 = u * u + v * v
    rho2 = f(2) * (dx * dx + dy * dy)
    rho = np.minimum(rho3, rho2)
    alpha = np.exp2(np.log2(o.astype(f)) - rho * f(0.5 * math.log2(math.e)))
    return rho3.astype(np.float64), rho2.astype(np.float64), np.minimum(alpha, f(0.99)).astype(np.float64)


def test_p21_fp32_error_model_bounds_rho_and_alpha():
    sc, cam = _degenerate_view()
    proj = oracle.project(sc, cam)
    off, ids, _ = oracle.bin_view(proj, cam)
    rng = np.random.default_rng(210)
    T = len(off) - 1
    tiles = np.flatnonzero(np.diff(off) > 0)
    # pairs: every listed entry of sampled tiles at four sampled pixels of the tile
    Ms, os_, xs, ys, degen = [], [], [], [], []
    s = np.exp(sc.log_scale.astype(np.float64))
    ratio = s.max(0) / s.min(0)
    tx = (cam.width + 15) // 16
    for t in rng.choice(tiles, size=min(120, tiles.size), replace=False):
        lst = ids[off[t]:off[t + 1]]
        for _ in range(4):
            px = (t % tx) * 16 + rng.integers(16) + 0.5
            py = (t // tx) * 16 + rng.integers(16) + 0.5
            Ms.append(proj["M"][lst])
            os_.append(proj["opacity"][lst])
            xs.append(np.full(lst.size, px))
            ys.append(np.full(lst.size, py))
            degen.append(ratio[lst] >= 50)
    M, o = np.concatenate(Ms), np.concatenate(os_)
    x, y, degen = np.concatenate(xs), np.concatenate(ys), np.concatenate(degen)
    ev = oracle.eval_pairs(M, o, np.stack([x, y], 1))
    r3, r2, a32 = _emulate(M, o, x, y)
    assert M.shape[0] > 50_000 and degen.sum() > 1000
    # rho3 where it decides: finite and not far beyond the cutoff (alpha >= 1e-6 o)
    live = np.isfinite(ev["rho3"]) & (np.minimum(ev["rho3"], ev["rho2"]) < 30) & np.isfinite(r3)
    e3 = np.abs(r3 - ev["rho3"])[live] / (ev["drho3"][live] / SAFETY)
    e2 = np.abs(r2 - ev["rho2"]) / (ev["drho2"] / SAFETY + 1e-300)
    ok = ev["alpha"] >= 1 / 255
    ea = np.abs(a32[ok] - ev["alpha"][ok]) / ev["alpha"][ok] / (ev["dalpha_rel"][ok] / SAFETY)
    assert live.sum() > 20_000 and ok.sum() > 5_000 and (degen & ok).sum() > 100
    print(f"P21 worst emulated/estimate: rho3 {e3.max():.3f}, rho2 {e2.max():.3f}, alpha {ea.max():.3f} "
          f"over {live.sum()} / {ok.sum()} pairs ({(degen & ok).sum()} degenerate)")
    assert e3.max() <= SLACK, f"rho3: emulated error {e3.max():.3f} x the model's estimate"
    assert e2[np.minimum(ev["rho3"], ev["rho2"]) < 30].max() <= SLACK
    assert ea.max() <= SLACK, f"alpha: emulated error {ea.max():.3f} x the model's estimate"


def test_p21_fp32_error_model_bounds_transmittance():
    """Along the blend of sampled pixels (the oracle's contributing fragments, in order), the emulated FP32
    transmittance T32 <- T32 (1 - alpha32) stays within the model's relative bound of T behind each
    fragment on pixels the model calls non-fragile."""
    sc, cam = _degenerate_view()
    proj = oracle.project(sc, cam)
    off, ids, _ = oracle.bin_view(proj, cam)
    rng = np.random.default_rng(211)
    tx = (cam.width + 15) // 16
    f = np.float32
    worst, frags, pixels = 0.0, 0, 0
    for t in rng.choice(np.flatnonzero(np.diff(off) > 8), size=60, replace=False):
        lst = ids[off[t]:off[t + 1]]
        for _ in range(3):
            x = (t % tx) * 16 + rng.integers(16) + 0.5
            y = (t // tx) * 16 + rng.integers(16) + 0.5
            fr, margin = oracle.blend_trace(proj, cam, lst, x, y)
            if margin < 1e-5 or len(fr) == 0:
                continue
            sid = fr[:, 0].astype(np.int64)
            _, _, a32 = _emulate(proj["M"][sid], proj["opacity"][sid], np.full(len(sid), x), np.full(len(sid), y))
            T32 = f(1)
            for k in range(len(sid)):
                assert a32[k] >= 1 / 255  # a contributing fragment stays one in FP32 on a non-fragile pixel
                T32 = f(T32 * (f(1) - f(a32[k])))
                T64 = fr[k, 2] * (1 - fr[k, 1])
                worst = max(worst, abs(float(T32) - T64) / T64 / (fr[k, 4] / SAFETY))
                frags += 1
            pixels += 1
    print(f"P21 worst emulated/estimate of T: {worst:.3f} over {frags} fragments of {pixels} pixels")
    assert pixels > 100 and frags > 1000
    assert worst <= SLACK, f"T: emulated error {worst:.3f} x the model's estimate"
