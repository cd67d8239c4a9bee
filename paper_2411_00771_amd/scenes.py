"""Seeded synthetic inputs: surfel sets, cameras, target images and request traces.

This module is shared by the HIP path, the CPU reference and the benchmark.  It
holds none of the rasterizer's arithmetic: it only draws random numbers and
builds camera poses.  The workloads stand in for the paper's aerial city
captures (Sec. 5.1: aerial images with the long side at 1,600 px, scenes of
0.3-2.7 km^2; Tab. 4: 5-10 M surfels per scene), which are not available here.

Layout (planar SoA, float32, what the C ABI consumes):
    mean[3][n], log_scale[2][n], quat[4][n] (w,x,y,z), opacity_logit[n],
    sh[(deg+1)^2][3][n]
Camera: world->camera ``Xc = R @ Xw + t`` (x right, y down, z forward), pinhole
intrinsics in pixels; pixel (i, j) samples (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TILE = 16


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float64, world -> camera
    t: np.ndarray  # (3,) float64
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    @property
    def tiles(self):
        return ((self.width + TILE - 1) // TILE, (self.height + TILE - 1) // TILE)

    def as_array(self) -> np.ndarray:
        """22 float64 values: W, H, fx, fy, cx, cy, R(9, row-major), t(3), znear, bg(3).

        All values are first rounded to float32, because the HIP path receives
        them as float32; both sides then see exactly the same camera.
        """
        v = [self.width, self.height, self.fx, self.fy, self.cx, self.cy]
        v += list(np.asarray(self.R, np.float64).reshape(-1)) + list(np.asarray(self.t, np.float64))
        v += [self.znear] + list(self.bg)
        a = np.array(v, np.float64)
        a[2:] = a[2:].astype(np.float32).astype(np.float64)
        return a


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def arrays(self):
        return dict(mean=self.mean, log_scale=self.log_scale, quat=self.quat,
                    opacity_logit=self.opacity_logit, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]), np.ascontiguousarray(self.log_scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]), np.ascontiguousarray(self.opacity_logit[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]), self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.mean.copy(), self.log_scale.copy(), self.quat.copy(),
                     self.opacity_logit.copy(), self.sh.copy(), self.sh_degree)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _sh_coeffs(rng, n, degree):
    k = (degree + 1) ** 2
    sh = np.empty((k, 3, n), np.float32)
    sh[0] = rng.uniform(0.0, 1.0, size=(3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.05, size=(k - 1, 3, n))
    return sh


def _random_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _rot_to_quat(Rm):
    """Rotation matrices (n, 3, 3) -> unit quaternions (4, n), w >= 0 (Shepperd's method)."""
    n = Rm.shape[0]
    q = np.empty((n, 4))
    tr = Rm[:, 0, 0] + Rm[:, 1, 1] + Rm[:, 2, 2]
    diag = np.stack([tr, Rm[:, 0, 0], Rm[:, 1, 1], Rm[:, 2, 2]], 1)
    k = np.argmax(diag, 1)
    for case in range(4):
        s = k == case
        if not np.any(s):
            continue
        R = Rm[s]
        if case == 0:
            r = np.sqrt(1.0 + tr[s]) * 2
            q[s] = np.stack([0.25 * r, (R[:, 2, 1] - R[:, 1, 2]) / r, (R[:, 0, 2] - R[:, 2, 0]) / r,
                             (R[:, 1, 0] - R[:, 0, 1]) / r], 1)
        elif case == 1:
            r = np.sqrt(1.0 + R[:, 0, 0] - R[:, 1, 1] - R[:, 2, 2]) * 2
            q[s] = np.stack([(R[:, 2, 1] - R[:, 1, 2]) / r, 0.25 * r, (R[:, 0, 1] + R[:, 1, 0]) / r,
                             (R[:, 0, 2] + R[:, 2, 0]) / r], 1)
        elif case == 2:
            r = np.sqrt(1.0 + R[:, 1, 1] - R[:, 0, 0] - R[:, 2, 2]) * 2
            q[s] = np.stack([(R[:, 0, 2] - R[:, 2, 0]) / r, (R[:, 0, 1] + R[:, 1, 0]) / r, 0.25 * r,
                             (R[:, 1, 2] + R[:, 2, 1]) / r], 1)
        else:
            r = np.sqrt(1.0 + R[:, 2, 2] - R[:, 0, 0] - R[:, 1, 1]) * 2
            q[s] = np.stack([(R[:, 1, 0] - R[:, 0, 1]) / r, (R[:, 0, 2] + R[:, 2, 0]) / r,
                             (R[:, 1, 2] + R[:, 2, 1]) / r, 0.25 * r], 1)
    q[q[:, 0] < 0] *= -1
    return q.T


# ----------------------------------------------------------------------------------------------
# Tiny scene: 4,096 surfels in [-1,1]^3, one camera at distance 3, 128x128, 60 deg FOV
# ----------------------------------------------------------------------------------------------

def tiny_scene(seed: int = 0, n: int = 4096, sh_degree: int = 3) -> Scene:
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, size=(3, n))
    ls = rng.uniform(math.log(0.005), math.log(0.05), size=(2, n))
    quat = _random_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    sh = _sh_coeffs(rng, n, sh_degree)
    return Scene(_f32(mean), _f32(ls), _f32(quat), _f32(logit), sh, sh_degree)


def tiny_camera(width: int = 128, height: int = 128, fov_deg: float = 60.0, dist: float = 3.0) -> Camera:
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, np.eye(3), np.array([0.0, 0.0, dist]))


def random_target(seed: int, width: int, height: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


# ----------------------------------------------------------------------------------------------
# Aerial city: fBm terrain + axis-aligned box buildings, surfels on the surfaces
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class City:
    L: float
    octaves: list          # (amplitude, wavelength, dirs (K,2), phases (K,))
    boxes: np.ndarray      # (B, 6): cx, cy, wx, wy, height, base z

    def height(self, x, y):
        h = np.zeros_like(np.asarray(x, np.float64))
        for amp, lam, dirs, ph in self.octaves:
            for d, p in zip(dirs, ph):
                h += amp * np.sin(2 * np.pi * (d[0] * x + d[1] * y) / lam + p) / math.sqrt(len(dirs))
        return h

    def grad(self, x, y):
        gx = np.zeros_like(np.asarray(x, np.float64))
        gy = np.zeros_like(gx)
        for amp, lam, dirs, ph in self.octaves:
            for d, p in zip(dirs, ph):
                c = amp * np.cos(2 * np.pi * (d[0] * x + d[1] * y) / lam + p) / math.sqrt(len(dirs)) * 2 * np.pi / lam
                gx += c * d[0]
                gy += c * d[1]
        return gx, gy


def make_city(seed: int, L: float = 1000.0, n_boxes: int = 200) -> City:
    rng = np.random.default_rng(seed)
    octaves = []
    amp, lam = 20.0, 400.0
    for _ in range(6):
        ang = rng.uniform(0, 2 * np.pi, size=4)
        dirs = np.stack([np.cos(ang), np.sin(ang)], 1)
        octaves.append((amp, lam, dirs, rng.uniform(0, 2 * np.pi, size=4)))
        amp *= 0.5
        lam *= 0.5
    city = City(L, octaves, np.zeros((0, 6)))
    bx = rng.uniform(-0.45 * L, 0.45 * L, size=(n_boxes, 2))
    wx = rng.uniform(10, 60, size=n_boxes)
    wy = rng.uniform(10, 60, size=n_boxes)
    hh = rng.uniform(10, 120, size=n_boxes)
    base = city.height(bx[:, 0], bx[:, 1])
    city.boxes = np.stack([bx[:, 0], bx[:, 1], wx, wy, hh, base], 1)
    return city


def _frames_from_normals(rng, nrm):
    """Orthonormal frames whose third column is the normal, with a uniform in-plane angle."""
    n = nrm.shape[0]
    helper = np.where(np.abs(nrm[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(helper, nrm)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nrm, e1)
    a = rng.uniform(0, 2 * np.pi, size=(n, 1))
    tu = np.cos(a) * e1 + np.sin(a) * e2
    tv = np.cross(nrm, tu)
    return np.stack([tu, tv, nrm], 2)  # columns


def city_scene(seed: int, n: int, L: float = 1000.0, sh_degree: int = 3,
               elongated_frac: float = 0.05, elong_range=(20.0, 50.0),
               lognormal_sigma: Optional[float] = None, city: Optional[City] = None) -> Scene:
    """Surfels sampled area-proportionally over terrain, roofs and walls.

    Scales: s = spacing * U[0.5, 1.5] per axis (or log-normal around the spacing
    when ``lognormal_sigma`` is given); a fraction ``elongated_frac`` gets an axis
    ratio drawn from ``elong_range`` with the area kept.
    """
    rng = np.random.default_rng(seed)
    city = city or make_city(seed, L)
    pos, nrm, spacing = _surface_samples(rng, city, n)

    perm = rng.permutation(n)
    pos, nrm = pos[perm], nrm[perm]
    Rm = _frames_from_normals(rng, nrm)
    quat = _rot_to_quat(Rm)

    if lognormal_sigma is None:
        su = spacing * rng.uniform(0.5, 1.5, size=n)
        sv = spacing * rng.uniform(0.5, 1.5, size=n)
    else:
        su = np.exp(rng.normal(math.log(spacing), lognormal_sigma, size=n))
        sv = np.exp(rng.normal(math.log(spacing), lognormal_sigma, size=n))
    el = rng.uniform(size=n) < elongated_frac
    ratio = rng.uniform(elong_range[0], elong_range[1], size=n)
    g = np.sqrt(su * sv)
    su = np.where(el, g * np.sqrt(ratio), su)
    sv = np.where(el, g / np.sqrt(ratio), sv)
    ls = np.log(np.stack([su, sv], 0))
    logit = rng.normal(0.0, 1.0, size=n)
    sh = _sh_coeffs(rng, n, sh_degree)
    return Scene(_f32(pos.T), _f32(ls), _f32(quat), _f32(logit), sh, sh_degree)


def _surface_samples(rng, city: City, n: int):
    """n positions (and normals) drawn area-proportionally over terrain, roofs and walls; the spacing
    sqrt(area / n)."""
    L = city.L
    B = city.boxes
    a_ter = L * L
    a_roof = B[:, 2] * B[:, 3]
    a_wall = 2 * (B[:, 2] + B[:, 3]) * B[:, 4]
    areas = np.array([a_ter, a_roof.sum(), a_wall.sum()])
    spacing = math.sqrt(areas.sum() / n)
    n_ter, n_roof, n_wall = rng.multinomial(n, areas / areas.sum())

    pos = np.empty((n, 3))
    nrm = np.empty((n, 3))
    # terrain
    x = rng.uniform(-L / 2, L / 2, size=n_ter)
    y = rng.uniform(-L / 2, L / 2, size=n_ter)
    gx, gy = city.grad(x, y)
    pos[:n_ter] = np.stack([x, y, city.height(x, y)], 1)
    nt = np.stack([-gx, -gy, np.ones_like(gx)], 1)
    nrm[:n_ter] = nt / np.linalg.norm(nt, axis=1, keepdims=True)
    # roofs
    o = n_ter
    bi = rng.choice(len(B), size=n_roof, p=a_roof / a_roof.sum())
    bb = B[bi]
    pos[o:o + n_roof] = np.stack([bb[:, 0] + (rng.uniform(size=n_roof) - 0.5) * bb[:, 2],
                                  bb[:, 1] + (rng.uniform(size=n_roof) - 0.5) * bb[:, 3],
                                  bb[:, 5] + bb[:, 4]], 1)
    nrm[o:o + n_roof] = np.array([0.0, 0.0, 1.0])
    # walls: 4 faces per box, weighted by face area
    o += n_roof
    face_a = np.stack([B[:, 3] * B[:, 4], B[:, 3] * B[:, 4], B[:, 2] * B[:, 4], B[:, 2] * B[:, 4]], 1).reshape(-1)
    fi = rng.choice(len(face_a), size=n_wall, p=face_a / face_a.sum())
    bi, face = fi // 4, fi % 4
    bb = B[bi]
    s = rng.uniform(size=n_wall) - 0.5
    hz = bb[:, 5] + rng.uniform(size=n_wall) * bb[:, 4]
    sx = np.where(face == 0, 0.5, np.where(face == 1, -0.5, s))
    sy = np.where(face == 2, 0.5, np.where(face == 3, -0.5, s))
    pos[o:] = np.stack([bb[:, 0] + sx * bb[:, 2], bb[:, 1] + sy * bb[:, 3], hz], 1)
    wn = np.zeros((n_wall, 3))
    wn[face == 0, 0] = 1
    wn[face == 1, 0] = -1
    wn[face == 2, 1] = 1
    wn[face == 3, 1] = -1
    nrm[o:] = wn
    return pos, nrm, spacing


def city_points(seed: int, n: int, city: City, noise: float = 0.05, chunk: int = 4_000_000) -> np.ndarray:
    """A synthetic ground-truth point cloud: points [3][n] (float32) on the city's surfaces with
    isotropic Gaussian noise of std ``noise`` (a scanner's), drawn in chunks to bound host memory."""
    rng = np.random.default_rng(seed)
    out = np.empty((3, n), np.float32)
    for a in range(0, n, chunk):
        k = min(chunk, n - a)
        pos, _, _ = _surface_samples(rng, city, k)
        out[:, a:a + k] = (pos + rng.normal(0.0, noise, size=pos.shape)).T
    return out


def _look_camera(pos, fwd, right, width, height, hfov_deg):
    fwd = fwd / np.linalg.norm(fwd)
    right = right - fwd * np.dot(right, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], 0)
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, R, -R @ pos)


def aerial_cameras(seed: int, city: City, count: int = 16, width: int = 1600, height: int = 1066,
                   hfov_deg: float = 60.0, alt=(100.0, 300.0), pitch_deg=(45.0, 90.0)) -> List[Camera]:
    """Cameras at (x, y) ~ U[-0.3L, 0.3L]^2, altitude above ground, pitch below the horizon, yaw uniform."""
    rng = np.random.default_rng(seed)
    L = city.L
    cams = []
    for _ in range(count):
        x, y = rng.uniform(-0.3 * L, 0.3 * L, size=2)
        z = float(city.height(np.array([x]), np.array([y]))[0]) + rng.uniform(*alt)
        th = math.radians(rng.uniform(*pitch_deg))
        yaw = rng.uniform(0, 2 * np.pi)
        fwd = np.array([math.cos(th) * math.cos(yaw), math.cos(th) * math.sin(yaw), -math.sin(th)])
        right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
        cams.append(_look_camera(np.array([x, y, z]), fwd, right, width, height, hfov_deg))
    return cams


def orbit_camera(rng, city: City, width: int, height: int, alt=(150.0, 400.0), radius=(0.25, 0.5),
                 hfov_deg: float = 60.0) -> Camera:
    L = city.L
    az = rng.uniform(0, 2 * np.pi)
    r = rng.uniform(*radius) * L
    pos = np.array([r * math.cos(az), r * math.sin(az), rng.uniform(*alt)])
    fwd = np.array([0.0, 0.0, float(city.height(np.array([0.0]), np.array([0.0]))[0])]) - pos
    right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    return _look_camera(pos, fwd, right, width, height, hfov_deg)


def nadir_grid_cameras(city: City, grid: int = 8, spacing: float = 200.0, alt: float = 250.0,
                       width: int = 3840, height: int = 2160, hfov_deg: float = 60.0) -> List[Camera]:
    cams = []
    off = (grid - 1) / 2.0
    for gy in range(grid):
        for gx in range(grid):
            x, y = (gx - off) * spacing, (gy - off) * spacing
            z = float(city.height(np.array([x]), np.array([y]))[0]) + alt
            cams.append(_look_camera(np.array([x, y, z]), np.array([0.0, 0.0, -1.0]),
                                     np.array([1.0, 0.0, 0.0]), width, height, hfov_deg))
    return cams


def perturbed(scene: Scene, seed: int, pos_sigma: float = 0.05, sh_sigma: float = 0.1) -> Scene:
    """A perturbed copy (target scenes: training against it gives structured gradients)."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    s.mean += (rng.normal(0, pos_sigma, size=s.mean.shape) * np.exp(s.log_scale).max(0)).astype(np.float32)
    s.sh[0] += rng.normal(0, sh_sigma, size=s.sh[0].shape).astype(np.float32)
    return s


def densify_inputs(seed: int, n: int, cand_frac: float = 0.05, remove_frac: float = 0.025):
    """Random inputs of a densification action over n surfels: a candidate mask (bit 4, the densify state's
    candidate bit), a removal mask (uint8 0/1) and the split children's standard-normal offsets
    z[n][2][2] (float32)."""
    rng = np.random.default_rng(seed)
    mask = np.where(rng.random(n) < cand_frac, 4, 0).astype(np.uint8) | rng.integers(0, 4, n).astype(np.uint8)
    remove = (rng.random(n) < remove_frac).astype(np.uint8)
    z = rng.standard_normal((n, 2, 2)).astype(np.float32)
    return mask, remove, z


def poisson_requests(seed: int, rate: float, duration: float, resolutions):
    """Arrival times (s) and a resolution index per request, open loop."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append((t, int(rng.integers(len(resolutions)))))
    return out


# ----------------------------------------------------------------------------------------------
# The five workloads (seed = workload index; cameras +1000, targets +2000, arrivals +3000)
# ----------------------------------------------------------------------------------------------

SERVE_RESOLUTIONS = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]


def morton_order(points: np.ndarray, bits: int = 21) -> np.ndarray:
    """Permutation that puts points [3][n] in 3-D Morton (octree) order, with cubic cells: the order in
    which octree-indexed point clouds are stored."""
    P = points.astype(np.float64)
    lo = P.min(1, keepdims=True)
    span = max(float((P.max(1, keepdims=True) - lo).max()), 1e-30)
    q = ((P - lo) / span * ((1 << bits) - 1)).astype(np.uint64)

    def spread(v):  # bit k of v -> bit 3k
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        return (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)

    code = spread(q[0]) | (spread(q[1]) << np.uint64(1)) | (spread(q[2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def crop_workload(n_points: int = 31_400_000, views: int = 958, width: int = 1920, height: int = 1080,
                  seed: int = 5):
    """Visibility-frequency crop-volume estimate of the evaluation protocol (Sec. 4): the scene it is
    quoted on covers 1.47 km^2 with 958 training views and 31.4 M ground-truth points, rendered at
    1080p.  Stand-in: a 1.47 km^2 synthetic city (L = 1212 m), a point cloud on its surfaces and
    aerial cameras over it.  The points are stored in 3-D Morton (octree) order."""
    city = make_city(seed, L=1212.0)
    pts = city_points(seed + 500, n_points, city)
    pts = np.ascontiguousarray(pts[:, morton_order(pts)])
    cams = aerial_cameras(seed + 1000, city, count=views, width=width, height=height)
    return dict(name=f"crop-{n_points // 1000}k-{views}v-{width}x{height}", points=pts, cameras=cams, city=city)


def workload(idx: int, n_override: Optional[int] = None):
    """Returns a dict describing one of the five synthetic workloads.

    0 tiny: 4,096 surfels, one 128x128 camera.
    1 aerial train step: 1 M surfels on a 1 km^2 city, 16 cameras at 1600x1066.
    2 batched training: the same generator at 4 M surfels, 8 views per launch.
    3 serving: 5 M surfels on a 1.6 km square city, Poisson requests at 200/s.
    4 largest: 10 M surfels, log-normal scales, 10 % elongated 50-1000.
    """
    if idx == 0:
        sc = tiny_scene(0, n_override or 4096)
        cam = tiny_camera()
        return dict(name="tiny-4096-128x128", scene=sc, cameras=[cam],
                    targets=[random_target(2000, cam.width, cam.height)])
    if idx in (1, 2):
        n = n_override or (1_000_000 if idx == 1 else 4_000_000)
        city = make_city(idx)
        sc = city_scene(idx, n, city=city)
        cams = aerial_cameras(idx + 1000, city, count=16 if idx == 1 else 8)
        return dict(name=f"aerial-{n // 1000}k-1600x1066", scene=sc, cameras=cams, city=city)
    if idx == 3:
        n = n_override or 5_000_000
        city = make_city(3, L=1600.0)
        sc = city_scene(3, n, L=1600.0, city=city)
        return dict(name=f"serve-{n // 1000}k-mixed", scene=sc, city=city,
                    requests=poisson_requests(3003, 200.0, 30.0, SERVE_RESOLUTIONS))
    if idx == 4:
        n = n_override or 10_000_000
        city = make_city(4)
        sc = city_scene(4, n, city=city, elongated_frac=0.10, elong_range=(50.0, 1000.0), lognormal_sigma=0.6)
        cams = aerial_cameras(1004, city, count=8)
        return dict(name=f"largest-{n // 1000}k", scene=sc, cameras=cams, city=city,
                    serve_cameras=nadir_grid_cameras(city))
    raise ValueError(idx)
