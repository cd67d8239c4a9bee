"""The host part of the crop-volume estimate (Sec. 4): the alpha shape of the kept ground points,
pinned to closed forms (areas of a square, an L shape, an annulus; the convex hull for alpha = inf)."""
import math

import numpy as np

from paper_2411_00771_amd.crop import alpha_shape


def _grid(x0, x1, y0, y1, step):
    xs = np.arange(x0, x1 + 1e-9, step)
    ys = np.arange(y0, y1 + 1e-9, step)
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()])


def test_square_grid_area_and_boundary():
    P = _grid(0, 10, 0, 10, 0.5)
    jitter = np.random.default_rng(0).uniform(-1e-6, 1e-6, P.shape)
    area, edges = alpha_shape(P + jitter, alpha=1.0)
    assert math.isclose(area, 100.0, rel_tol=1e-5)
    # the boundary runs along the square's perimeter: 4 x 20 unit steps of 0.5
    assert len(edges) == 80


def test_infinite_alpha_is_the_convex_hull():
    from scipy.spatial import ConvexHull
    P = np.random.default_rng(1).normal(size=(2, 500))
    area, _ = alpha_shape(P, alpha=np.inf)
    assert math.isclose(area, ConvexHull(P.T).volume, rel_tol=1e-12)


def test_l_shape_and_annulus():
    rng = np.random.default_rng(2)
    L = np.concatenate([_grid(0, 10, 0, 4, 0.25), _grid(0, 4, 4.25, 10, 0.25)], axis=1)
    # the two blocks plus the corner triangle (4, 4), (4.25, 4), (4, 4.25) (circumradius 0.177 < alpha)
    area, _ = alpha_shape(L + rng.uniform(-1e-6, 1e-6, L.shape), alpha=0.3)
    assert math.isclose(area, 10 * 4 + 4 * 6 + 0.5 * 0.25 * 0.25, rel_tol=1e-6)
    # annulus 3 <= r <= 5, dense: the hole is excluded for a small alpha, filled for alpha = inf
    r = np.sqrt(rng.uniform(9, 25, 40000))
    t = rng.uniform(0, 2 * np.pi, 40000)
    A = np.stack([r * np.cos(t), r * np.sin(t)])
    area, _ = alpha_shape(A, alpha=0.3)
    assert abs(area - math.pi * (25 - 9)) < 0.02 * math.pi * 16
    area_inf, _ = alpha_shape(A, alpha=np.inf)
    assert area_inf > math.pi * 24


def test_degenerate_inputs():
    assert alpha_shape(np.zeros((2, 0)), 1.0)[0] == 0.0
    assert alpha_shape(np.array([[0.0, 1.0], [0.0, 1.0]]), 1.0)[0] == 0.0
