"""Seeded synthetic inputs: multi-level Gaussian scenes, cameras and request streams.

This module draws random numbers and lays them out; it holds none of the
rasteriser's arithmetic (no projection, coverage, selection or blending).  It is
the only module that both the HIP path and the CPU oracle's tests use.

Scenes follow the representation of the paper's preliminaries (Sec. 3.1): every
Gaussian has a centre, a covariance built from a per-axis scale and a rotation
quaternion, a density (opacity) and colour, here spherical-harmonic features
(Supplementary, average pooling).  Each Gaussian carries a level tag (Sec. 4.1:
four levels for 1x/4x/16x/64x downsampling), stored 0-based with level 0 the
finest, and the stored pixel-coverage range S^max/S^min read by selective
rendering (Sec. 4.1 on selective rendering).

Layout (planar fp32, one plane per component, length n each):
  means  [3][n]  x, y, z
  scales [3][n]  linear per-axis standard deviations (> 0)
  quats  [4][n]  w, x, y, z (any non-zero length; normalised by the renderer)
  opacity[n]     density sigma in [0, 1)
  sh     [(D+1)^2 * 3][n]  plane (j*3 + c) holds SH coefficient j of channel c
  level  [n]     uint8, 0 = finest
  s_max, s_min [n]  stored coverage range; (0, +inf) until calibrated

Workload recipes (the paper's datasets are not available; these synthetic
stand-ins have the structure stated for each workload):
  * single-level scene, 10,000 Gaussians, means U[-1,1]^3, log-scale N(-3.5,0.5),
    opacity sigmoid(N(0,1)), SH degree 0 with DC U[0,1]; camera at distance 3,
    128x128, f=150.
  * 4-level scene, level l holds 400k/4^l Gaussians with log-scale mean
    -4.5+1.4 l; 75% of level 0 from 8 clustered blobs; SH degree 3 N(0,0.2);
    camera 1600x1064, f=1875.
  * 3M / 6M Gaussian scenes (4 / 5 levels, counts proportional to 4^-l), uniform
    means, the same per-level size law, SH degree 3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Scene", "Camera", "lookat_camera", "sphere_poses", "make_scene",
    "single_level_scene", "four_level_scene", "large_scene", "level_counts",
    "calibration_cameras", "request_stream", "open_ranges", "save_scene",
    "load_scene", "reset_ranges", "random_target",
]


@dataclasses.dataclass
class Scene:
    n: int
    sh_degree: int
    n_levels: int
    means: np.ndarray      # float32 [3, n]
    scales: np.ndarray     # float32 [3, n]
    quats: np.ndarray      # float32 [4, n]
    opacity: np.ndarray    # float32 [n]
    sh: np.ndarray         # float32 [(D+1)^2*3, n]
    level: np.ndarray      # uint8 [n]
    s_max: np.ndarray      # float32 [n]
    s_min: np.ndarray      # float32 [n]

    def copy(self) -> "Scene":
        return Scene(**{f.name: (getattr(self, f.name).copy()
                                 if isinstance(getattr(self, f.name), np.ndarray)
                                 else getattr(self, f.name))
                        for f in dataclasses.fields(self)})

    def subset(self, idx: np.ndarray) -> "Scene":
        idx = np.asarray(idx)
        return Scene(n=int(idx.size), sh_degree=self.sh_degree, n_levels=self.n_levels,
                     means=np.ascontiguousarray(self.means[:, idx]),
                     scales=np.ascontiguousarray(self.scales[:, idx]),
                     quats=np.ascontiguousarray(self.quats[:, idx]),
                     opacity=np.ascontiguousarray(self.opacity[idx]),
                     sh=np.ascontiguousarray(self.sh[:, idx]),
                     level=np.ascontiguousarray(self.level[idx]),
                     s_max=np.ascontiguousarray(self.s_max[idx]),
                     s_min=np.ascontiguousarray(self.s_min[idx]))


@dataclasses.dataclass
class Camera:
    R: np.ndarray   # float32 [9], row-major world->camera rotation (OpenCV axes)
    t: np.ndarray   # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


def lookat_camera(position: Sequence[float], width: int, height: int, focal: float,
                  target: Sequence[float] = (0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at `position` looking at `target`; x right, y down (world +y
    is down), z forward.  Principal point at the image centre."""
    c = np.asarray(position, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    down = np.array([0.0, 1.0, 0.0])
    if abs(float(np.dot(down, z))) > 0.999:
        down = np.array([0.0, 0.0, 1.0])
    x = np.cross(down, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])            # rows = camera axes in world coords
    t = -R @ c
    return Camera(R=R.astype(np.float32).reshape(9), t=t.astype(np.float32),
                  fx=float(focal), fy=float(focal), cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height))


def sphere_poses(n: int, seed: int, rmin: float, rmax: float) -> List[np.ndarray]:
    """`n` camera positions: uniform direction on the unit sphere, radius U[rmin, rmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = rng.uniform(rmin, rmax)
        out.append(d * r)
    return out


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def level_counts(total: int, n_levels: int) -> List[int]:
    """Split `total` Gaussians over levels proportionally to 4^-l (largest
    remainder rounding, so the counts sum to `total`)."""
    w = np.array([4.0 ** -l for l in range(n_levels)])
    exact = total * w / w.sum()
    base = np.floor(exact).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return [int(v) for v in base]


def make_scene(counts: Sequence[int], seed: int, sh_degree: int,
               logscale_mean: Sequence[float], logscale_std: float = 0.5,
               blob_fraction0: float = 0.0, n_blobs: int = 8,
               sh_std: float = 0.2, dc_uniform: bool = False,
               extent: float = 1.0) -> Scene:
    """Generic multi-level generator.  Level l has counts[l] Gaussians with
    log-scale ~ N(logscale_mean[l], logscale_std) per axis; a fraction
    `blob_fraction0` of level 0 is drawn from `n_blobs` isotropic blobs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = len(counts)
    n = int(sum(counts))
    K = (sh_degree + 1) ** 2
    means = np.empty((3, n), np.float64)
    logs = np.empty((3, n), np.float64)
    level = np.empty(n, np.uint8)
    blobs = rng.uniform(-0.8 * extent, 0.8 * extent, size=(n_blobs, 3))
    o = 0
    for l, c in enumerate(counts):
        if l == 0 and blob_fraction0 > 0:
            nb = int(round(c * blob_fraction0))
            which = rng.integers(0, n_blobs, size=nb)
            pb = blobs[which] + rng.normal(0.0, 0.08 * extent, size=(nb, 3))
            pu = rng.uniform(-extent, extent, size=(c - nb, 3))
            p = np.clip(np.concatenate([pb, pu]), -extent, extent)
            p = p[rng.permutation(c)]
        else:
            p = rng.uniform(-extent, extent, size=(c, 3))
        means[:, o:o + c] = p.T
        logs[:, o:o + c] = rng.normal(logscale_mean[l], logscale_std, size=(3, c))
        level[o:o + c] = l
        o += c
    quats = _unit_quats(rng, n)
    opacity = _sigmoid(rng.standard_normal(n)).astype(np.float32)
    if dc_uniform:
        sh = np.zeros((K * 3, n), np.float32)
        sh[0:3] = rng.uniform(0.0, 1.0, size=(3, n))
    else:
        sh = rng.normal(0.0, sh_std, size=(K * 3, n)).astype(np.float32)
    return Scene(n=n, sh_degree=sh_degree, n_levels=L,
                 means=means.astype(np.float32),
                 scales=np.exp(logs).astype(np.float32),
                 quats=quats, opacity=opacity, sh=sh, level=level,
                 s_max=np.zeros(n, np.float32),
                 s_min=np.full(n, np.inf, np.float32))


def single_level_scene(n: int = 10_000, seed: int = 1) -> Scene:
    """The 10k single-level workload: log-scale N(-3.5, 0.5), SH degree 0, DC U[0,1]."""
    return make_scene([n], seed, 0, [-3.5], dc_uniform=True)


def four_level_scene(seed: int = 2, per_level0: int = 400_000) -> Scene:
    """The 4-level workload: level l holds per_level0/4^l Gaussians, log-scale mean
    -4.5+1.4l, 75% of level 0 in 8 blobs, SH degree 3 ~ N(0, 0.2)."""
    counts = [per_level0 // 4 ** l for l in range(4)]
    return make_scene(counts, seed, 3, [-4.5 + 1.4 * l for l in range(4)],
                      blob_fraction0=0.75)


def large_scene(total: int, n_levels: int, seed: int) -> Scene:
    """3M / 6M workloads: counts proportional to 4^-l, uniform means, per-level
    log-scale mean -4.5+1.4l, SH degree 3 ~ N(0, 0.2)."""
    return make_scene(level_counts(total, n_levels), seed, 3,
                      [-4.5 + 1.4 * l for l in range(n_levels)])


def calibration_cameras(seed: int, width: int, height: int, focal: float,
                        k: int = 8, radius: float = 3.0) -> List[Camera]:
    """K look-at cameras on a sphere of fixed radius, used to establish the stored
    coverage range of every level before rendering."""
    return [lookat_camera(p, width, height, focal)
            for p in sphere_poses(k, seed, radius, radius)]


def request_stream(seed: int = 4, n: int = 512, rate_hz: float = 200.0,
                   rmin: float = 2.0, rmax: float = 12.0,
                   downscales: Sequence[int] = (1, 2, 4, 8, 16, 32, 64, 128),
                   width: int = 1920, height: int = 1080, focal: float = 2250.0):
    """Poisson stream of render requests: (arrival_s, camera, downscale)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    ds = rng.choice(np.asarray(downscales), size=n)
    poses = sphere_poses(n, seed + 1000, rmin, rmax)
    return [(float(arrivals[i]), lookat_camera(poses[i], width, height, focal), int(ds[i]))
            for i in range(n)]


def random_target(seed: int, height: int, width: int) -> np.ndarray:
    """Seeded U[0,1] target image [H][W][3] fp32 for an L2 loss."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(height, width, 3)).astype(np.float32)


def open_ranges(scene: Scene) -> Scene:
    """Copy of `scene` with S^max=+inf and S^min=0, under which every Gaussian in
    front of the camera passes selection."""
    s = scene.copy()
    s.s_max[:] = np.inf
    s.s_min[:] = 0.0
    return s


def reset_ranges(scene: Scene) -> Scene:
    """Copy of `scene` with the un-calibrated range (0, +inf)."""
    s = scene.copy()
    s.s_max[:] = 0.0
    s.s_min[:] = np.inf
    return s


def save_scene(path: str, scene: Scene) -> None:
    np.savez(path, **{f.name: np.asarray(getattr(scene, f.name))
                      for f in dataclasses.fields(scene)})


def load_scene(path: str) -> Scene:
    with np.load(path, allow_pickle=False) as z:
        kw = {}
        for f in dataclasses.fields(Scene):
            v = z[f.name]
            kw[f.name] = int(v) if v.ndim == 0 else v
        return Scene(**kw)
