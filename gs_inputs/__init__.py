"""Seeded synthetic inputs for the Gaussian rasterizer: scenes, cameras, masks, targets.

This module only draws numbers and lays them out; it holds none of the
rasterizer's arithmetic, so the FP64 oracle and the HIP path can both consume
it without sharing code.  All draws use ``numpy.random.Generator(PCG64(seed))``
in a fixed order, so a (recipe, seed) pair names one exact input.

Layouts (structure of arrays, float32, C-contiguous):
  means   [3][N]          world positions
  scales  [3][N]          activated (positive) per-axis standard deviations
  quats   [4][N]          (w, x, y, z), not normalised
  opacity [N]             activated opacity in (0, 1)
  sh      [16][3][N]      real-SH coefficients, plane index k*3 + channel

Cameras are world->camera rigid transforms in the OpenCV convention
(x right, y down, z forward) with a pinhole intrinsic; pixel (px, py) samples
the continuous image point (px + 0.5, py + 0.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

SH_COEFFS = 16


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def subset(self, idx: np.ndarray) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]),
                     self.sh_degree)

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.means, self.scales, self.quats, self.opacity, self.sh))


@dataclasses.dataclass
class Camera:
    R: np.ndarray        # [3,3] float32, world -> camera rotation
    t: np.ndarray        # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_tuple(self):
        return (self.R, self.t, self.fx, self.fy, self.cx, self.cy, self.width, self.height)


def _attributes(g: np.random.Generator, n: int, log_scale_mu: float, log_scale_sd: float):
    scales = np.exp(g.normal(log_scale_mu, log_scale_sd, size=(3, n))).astype(np.float32)
    quats = g.normal(0.0, 1.0, size=(4, n))
    quats /= np.linalg.norm(quats, axis=0, keepdims=True)
    quats = quats.astype(np.float32)
    opacity = (1.0 / (1.0 + np.exp(-g.normal(0.0, 1.0, size=n)))).astype(np.float32)
    sh = np.empty((SH_COEFFS, 3, n), dtype=np.float32)
    sh[0] = g.normal(0.5, 0.2, size=(3, n))
    sh[1:] = g.normal(0.0, 0.05, size=(SH_COEFFS - 1, 3, n))
    return scales, quats, opacity, sh


def uniform_cube_scene(n: int, seed: int, half: float = 1.0,
                       log_scale_mu: float = -3.5, log_scale_sd: float = 0.5) -> Scene:
    """Means uniform in [-half, half]^3; the small-scene recipe (4,096 Gaussians)."""
    g = rng(seed)
    means = g.uniform(-half, half, size=(3, n)).astype(np.float32)
    scales, quats, opacity, sh = _attributes(g, n, log_scale_mu, log_scale_sd)
    return Scene(means, scales, quats, opacity, sh)


def surface_scene(n: int, seed: int, centre_half: float = 2.0, n_surfaces: int = 20,
                  noise: float = 0.02, log_scale_mu: float = -5.0, log_scale_sd: float = 0.7) -> Scene:
    """Means on random spheres / square plane patches plus Gaussian noise.

    Each surface is a sphere or a plane patch with probability 1/2, centre
    uniform in [-centre_half, centre_half]^3, radius U(0.5, 3) (a plane patch is a
    square of half-side = radius with a random unit normal).  Points are spread
    evenly over the surfaces (the first n % n_surfaces surfaces get one more).
    """
    g = rng(seed)
    counts = np.full(n_surfaces, n // n_surfaces, dtype=np.int64)
    counts[: n % n_surfaces] += 1
    parts = []
    for s in range(n_surfaces):
        kind_sphere = g.uniform() < 0.5
        centre = g.uniform(-centre_half, centre_half, size=3)
        radius = g.uniform(0.5, 3.0)
        m = int(counts[s])
        if kind_sphere:
            d = g.normal(0.0, 1.0, size=(3, m))
            d /= np.linalg.norm(d, axis=0, keepdims=True)
            pts = centre[:, None] + radius * d
        else:
            nrm = g.normal(0.0, 1.0, size=3)
            nrm /= np.linalg.norm(nrm)
            helper = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            e1 = np.cross(nrm, helper)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(nrm, e1)
            ab = g.uniform(-radius, radius, size=(2, m))
            pts = centre[:, None] + e1[:, None] * ab[0] + e2[:, None] * ab[1]
        parts.append(pts)
    means = np.concatenate(parts, axis=1)
    means += g.normal(0.0, noise, size=means.shape)
    means = means.astype(np.float32)
    scales, quats, opacity, sh = _attributes(g, n, log_scale_mu, log_scale_sd)
    return Scene(np.ascontiguousarray(means), scales, quats, opacity, sh)


def look_at(eye: Sequence[float], target: Sequence[float], width: int, height: int,
            fov_x_deg: float = 60.0) -> Camera:
    """Pinhole camera at ``eye`` looking at ``target``; horizontal field of view.

    z_c = normalize(target - eye), x_c = normalize(z_c x up), y_c = z_c x x_c with
    up = +y (or +z when the view direction is almost vertical); fx = fy =
    (W/2)/tan(fov_x/2); principal point at the image centre.
    """
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    zc = target - eye
    zc /= np.linalg.norm(zc)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(zc @ up)) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    xc = np.cross(zc, up)
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R, t, float(np.float32(f)), float(np.float32(f)),
                  float(width) / 2.0, float(height) / 2.0, int(width), int(height))


def sphere_cameras(count: int, radius: float, resolutions: Sequence[Tuple[int, int]],
                   seed: int, fov_x_deg: float = 60.0) -> List[Camera]:
    """``count`` cameras at seeded directions on a sphere, looking at the origin."""
    g = rng(seed)
    cams = []
    for k in range(count):
        d = g.normal(0.0, 1.0, size=3)
        d /= np.linalg.norm(d)
        w, h = resolutions[k % len(resolutions)]
        cams.append(look_at(radius * d, (0.0, 0.0, 0.0), w, h, fov_x_deg))
    return cams


def bernoulli_mask(n: int, p: float, seed: int) -> np.ndarray:
    return (rng(seed).uniform(size=n) < p).astype(np.uint8)


def importance_like(views: int, n: int, seed: int, zero_fraction: float = 0.4, sigma: float = 2.0) -> np.ndarray:
    """[views, n] float32: heavy-tailed non-negative sums of blend weights, with
    a fraction of exact zeros (Gaussians that reach no pixel of the view)."""
    g = rng(seed)
    v = g.lognormal(mean=0.0, sigma=sigma, size=(views, n))
    v[g.uniform(size=(views, n)) < zero_fraction] = 0.0
    return v.astype(np.float32)


def wmax_like(n: int, seed: int, clamp_fraction: float = 0.2, alpha_max: float = 0.99):
    """(area[n] uint32, wmax[n] float32): maximum blend weights in (0, alpha_max],
    a fraction exactly alpha_max (the first Gaussian of a pixel at the opacity
    clamp), and argmax areas that are zero for about half of the Gaussians."""
    g = rng(seed)
    w = g.beta(2.0, 5.0, size=n) * alpha_max
    w[g.uniform(size=n) < clamp_fraction] = alpha_max
    area = np.where(g.uniform(size=n) < 0.5, 0, g.geometric(0.05, size=n)).astype(np.uint32)
    return area, w.astype(np.float32)


def exponential_draws(n: int, seed: int) -> np.ndarray:
    """Exp(1) variates, float32 (the random draws of weighted sampling)."""
    return rng(seed).exponential(size=n).astype(np.float32)


def uniform_draws(n: int, seed: int) -> np.ndarray:
    """U[0, 1) variates, float32."""
    return rng(seed).uniform(size=n).astype(np.float32)


def normal_draws(shape, seed: int) -> np.ndarray:
    """N(0, 1) variates, float32 (the position draws of the split)."""
    return rng(seed).standard_normal(size=shape).astype(np.float32)


def gradient_stats_like(n: int, seed: int, unseen_fraction: float = 0.2):
    """(norm_sum[n] float32, count[n] uint32): accumulated screen-gradient
    norms over up to 16 views, log-normal per view, some rows never seen."""
    g = rng(seed)
    count = g.integers(1, 17, size=n).astype(np.uint32)
    count[g.uniform(size=n) < unseen_fraction] = 0
    norm_sum = (count * np.exp(g.normal(-8.0, 1.5, size=n))).astype(np.float32)
    return norm_sum, count


def depth_map_like(pixels: int, seed: int, near: float = 0.5, far: float = 12.0, empty_fraction: float = 0.2):
    """(depth[P] float32, imax[P] int32, hit[P] uint8): a rendered depth map
    with a fraction of empty pixels (imax = -1, depth 0) and rays that miss
    their max-weight ellipsoid (hit = 0)."""
    g = rng(seed)
    depth = g.uniform(near, far, size=pixels).astype(np.float32)
    imax = g.integers(0, 1 << 20, size=pixels).astype(np.int32)
    empty = g.uniform(size=pixels) < empty_fraction
    imax[empty] = -1
    depth[empty] = 0.0
    hit = ((g.uniform(size=pixels) < 0.85) & ~empty).astype(np.uint8)
    return depth, imax, hit


def uniform_image(channels: int, pixels: int, seed: int) -> np.ndarray:
    return rng(seed).uniform(0.0, 1.0, size=(channels, pixels)).astype(np.float32)


def normal_image(channels: int, pixels: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return (scale * rng(seed).normal(0.0, 1.0, size=(channels, pixels))).astype(np.float32)


# ----------------------------------------------------------------------------------
# Named workloads (sizes and distributions of the paper-scale experiments)
# ----------------------------------------------------------------------------------
MULTIVIEW_RESOLUTIONS = [(640, 480), (800, 600), (1024, 768), (1280, 720),
                         (1280, 960), (1440, 1080), (1600, 900), (1600, 1200)]
SERVING_SCENE_SIZES = [200_000, 500_000, 1_000_000, 1_500_000, 2_000_000, 2_500_000,
                       3_000_000, 3_000_000]
SERVING_RESOLUTIONS = [(800, 800), (1280, 720), (1920, 1080)]


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cameras: List[Camera]
    active: np.ndarray | None = None


def small_cube(seed: int = 0, n: int = 4096, width: int = 128, height: int = 128) -> Workload:
    """4,096 Gaussians in [-1,1]^3, one 128x128 view from (0,0,4), fov 60 deg."""
    sc = uniform_cube_scene(n, seed)
    cam = look_at((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), width, height)
    return Workload("small_cube_4k_128px", sc, [cam])


def heavy_tiles(seed: int = 0, n: int = 40_000, width: int = 64, height: int = 48,
                opacity=(0.01, 0.05), distance: float = 2.5) -> Workload:
    """Dense, faint cube filling a small view: every 16x16 tile holds a list of
    a few thousand entries and pixels composite hundreds of them before the
    transmittance stop (default opacity U(0.01, 0.05)), the regime of the heavy tiles
    of a full-size scene at a size the oracle renders in seconds."""
    sc = uniform_cube_scene(n, seed)
    sc.opacity = rng(seed + 1).uniform(opacity[0], opacity[1], size=n).astype(np.float32)
    cam = look_at((0.0, 0.0, distance), (0.0, 0.0, 0.0), width, height)
    return Workload("heavy_tiles_40k_64x48", sc, [cam])


def elongated_cube(seed: int = 0, n: int = 3000, width: int = 160, height: int = 128,
                   stretch: float = 12.0) -> Workload:
    """Cube scene whose Gaussians are needles (one axis `stretch` times the
    others, random orientation): their screen ellipses are long and tilted,
    so many tiles of their bounding boxes lie outside the alpha >= 1/255
    region (the case tile culling at emission addresses)."""
    sc = uniform_cube_scene(n, seed, log_scale_mu=-3.8)
    sc.scales = sc.scales.copy()
    sc.scales[0] *= np.float32(stretch)
    cam = look_at((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), width, height)
    return Workload("elongated_cube_3k", sc, [cam])


def training_view(seed: int = 1, n: int = 500_000) -> Workload:
    """500k surface-sampled Gaussians, one 1245x825 view from a radius-6 sphere."""
    sc = surface_scene(n, seed, centre_half=2.0)
    cams = sphere_cameras(1, 6.0, [(1245, 825)], seed + 1000)
    return Workload("surfaces_500k_1245x825", sc, cams)


def large_scene(seed: int = 2, n: int = 3_000_000, radius: float = 30.0,
                active_p: float = 0.25) -> Workload:
    """3M surface-sampled Gaussians over [-10,10]^3, one 1920x1080 view, 25% active."""
    sc = surface_scene(n, seed, centre_half=10.0)
    cams = sphere_cameras(1, radius, [(1920, 1080)], seed + 1000)
    return Workload("surfaces_3M_1920x1080", sc, cams, bernoulli_mask(n, active_p, seed + 2000))


def multiview(seed: int = 3, n: int = 1_000_000, views: int = 16) -> Workload:
    """1M surface-sampled Gaussians, 16 views of mixed resolution on a radius-6 sphere."""
    sc = surface_scene(n, seed, centre_half=2.0)
    res = [r for r in MULTIVIEW_RESOLUTIONS for _ in range(2)][:views]
    cams = sphere_cameras(views, 6.0, res, seed + 1000)
    return Workload("surfaces_1M_16views_mixed", sc, cams)
