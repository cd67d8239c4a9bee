"""Seeded generators: determinism, shapes and the stated value distributions."""
import math

import numpy as np

from paper_2411_00771_amd import scenes


def test_tiny_deterministic_and_shaped():
    a, b = scenes.tiny_scene(0), scenes.tiny_scene(0)
    for k in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
        assert getattr(a, k).dtype == np.float32 and getattr(a, k).flags.c_contiguous
    assert a.mean.shape == (3, 4096) and a.sh.shape == (16, 3, 4096)
    assert a.mean.min() >= -1 and a.mean.max() <= 1
    assert a.log_scale.min() >= math.log(0.005) - 1e-6 and a.log_scale.max() <= math.log(0.05) + 1e-6
    assert np.allclose(np.linalg.norm(a.quat, axis=0), 1, atol=1e-6)
    assert 0 <= a.sh[0].min() and a.sh[0].max() <= 1
    assert abs(a.sh[1:].std() - 0.05) < 0.005
    cam = scenes.tiny_camera()
    assert abs(cam.fx - 64 / math.tan(math.radians(30))) < 1e-9


def test_city_elongated_fraction_and_cameras():
    city = scenes.make_city(1)
    sc = scenes.city_scene(1, 20000, city=city)
    s = np.exp(sc.log_scale.astype(np.float64))
    ratio = s.max(0) / s.min(0)
    frac = (ratio > 20).mean()
    assert 0.04 < frac < 0.06
    cams = scenes.aerial_cameras(1001, city, count=16)
    for c in cams:
        assert (c.width, c.height) == (1600, 1066)
        R = c.R
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        fwd = R[2]
        pitch = math.degrees(math.asin(-fwd[2]))
        assert 45 - 1e-6 <= pitch <= 90 + 1e-6
        C = c.center
        ground = float(city.height(np.array([C[0]]), np.array([C[1]]))[0])
        assert 100 - 1e-6 <= C[2] - ground <= 300 + 1e-6


def test_requests_poisson_rate():
    req = scenes.poisson_requests(3003, 200.0, 30.0, scenes.SERVE_RESOLUTIONS)
    assert abs(len(req) / 30.0 - 200) < 10
    t = np.array([r[0] for r in req])
    assert np.all(np.diff(t) > 0)
