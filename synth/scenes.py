"""Seeded synthetic Gaussian scenes and pinhole cameras.

Every array is drawn with ``numpy.random.default_rng(seed)`` (PCG64) in float64
and cast once to float32; the oracle and the GPU path read the same bytes.

Scene layout (array of structures on the host, one row per Gaussian):
  means           (N, 3)  world-space centres
  log_scales      (N, 3)  per-axis log standard deviations
  quats           (N, 4)  rotation quaternion, (w, x, y, z), not normalised
  opacity_logits  (N,)    opacity before the logistic activation
  sh              (N, K, 3) spherical-harmonic colour coefficients,
                  K = (degree + 1)^2, coefficient index l*l + l + m

Camera: OpenCV axes (x right, y down, z forward); ``world_to_cam`` is the
row-major 3x4 matrix [R | t] with p_cam = R p_world + t; intrinsics in pixels.
World "up" is -y, so an orbit elevation lifts the camera towards -y.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

# The degree-0 SH basis value, used only to encode a target RGB in [0, 1] as a
# DC coefficient for the small parity scene: rgb = dc * Y00 + 1/2.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)


@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # (3, 4) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def scene_small(n: int = 2000, seed: int = 0) -> Scene:
    """Small parity scene: means U[-1,1]^3, log-scales N(-3,0.5), random
    quaternions, opacity logits N(0,1.5), SH degree 0 holding rgb ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(0.0, 1.5, size=(n,))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = ((rgb - 0.5) / _Y00).reshape(n, 1, 3)
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 0)


def scene_small_sh3(n: int = 400, seed: int = 0) -> Scene:
    """scene_small's layout with larger footprints (centres x 0.6, log-scales
    + 0.8) and SH degree 3: the DC term holds rgb ~ U[0, 1], the 15 higher
    coefficients per channel are N(0, 0.3). Float64 arrays, so that finite
    differences see the exact inputs."""
    base = scene_small(n, seed=seed)
    rng = np.random.default_rng(seed + 100)
    sh = np.zeros((n, 16, 3))
    sh[:, :1, :] = base.sh
    sh[:, 1:, :] = rng.normal(0.0, 0.3, size=(n, 15, 3))
    f64 = lambda a: np.asarray(a, dtype=np.float64).copy()
    return Scene(f64(base.means) * 0.6, f64(base.log_scales) + 0.8, f64(base.quats), f64(base.opacity_logits),
                 sh, 3)


def scene_needles(n: int = 1500, seed: int = 0) -> Scene:
    """Stress scene for the FP32 precision of the blend: means U[-1,1]^3,
    one log-scale N(-1.5,0.5) and two N(-6,0.7) per Gaussian (axis ratios
    ~10^2 to 10^3, so projected footprints are long thin needles at every
    angle), random quaternions, opacity logits N(1,2), rgb ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = rng.normal(-6.0, 0.7, size=(n, 3))
    log_scales[np.arange(n), rng.integers(0, 3, size=n)] = rng.normal(-1.5, 0.5, size=n)
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(1.0, 2.0, size=(n,))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = ((rgb - 0.5) / _Y00).reshape(n, 1, 3)
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 0)


def _cluster_means(rng, n, n_clusters, box, std_lo, std_hi, log_uniform):
    centers = rng.uniform(-box, box, size=(n_clusters, 3))
    if log_uniform:
        stds = np.exp(rng.uniform(math.log(std_lo), math.log(std_hi), size=(n_clusters, 3)))
    else:
        stds = rng.uniform(std_lo, std_hi, size=(n_clusters, 3))
    rots = Rotation.random(n_clusters, random_state=rng).as_matrix()  # (C, 3, 3)
    which = rng.integers(0, n_clusters, size=n)
    local = rng.normal(0.0, 1.0, size=(n, 3)) * stds[which]
    pts = centers[which] + np.einsum("nij,nj->ni", rots[which], local)
    return np.clip(pts, -box, box)


def _sh_coeffs(rng, n, degree, dc_std=0.5, hi_std=0.05):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = rng.normal(0.0, dc_std, size=(n, 3))
    for c in range(1, k):
        sh[:, c, :] = rng.normal(0.0, hi_std, size=(n, 3))
    return sh


def scene_clusters(n: int = 1_000_000, seed: int = 0, sh_degree: int = 3,
                   n_clusters: int = 64, box: float = 10.0) -> Scene:
    """Headline scene: means from a mixture of anisotropic Gaussian clusters in
    a 20 m box (cluster axis std log-uniform in [0.5, 3] m under a random
    rotation), log-scales N(-4,1), opacity logits N(0,2), SH DC N(0,0.5) and
    higher bands N(0,0.05)."""
    rng = np.random.default_rng(seed)
    means = _cluster_means(rng, n, n_clusters, box, 0.5, 3.0, True)
    log_scales = rng.normal(-4.0, 1.0, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(0.0, 2.0, size=(n,))
    sh = _sh_coeffs(rng, n, sh_degree)
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), sh, sh_degree)


def scene_heavy(n: int = 3_000_000, seed: int = 0, sh_degree: int = 3,
                dense_frac: float = 0.2, box: float = 10.0) -> Scene:
    """Load-imbalanced scene: (1 - dense_frac) of the Gaussians from the
    cluster generator and dense_frac from 8 tight clusters (axis std U[0.1,0.4]
    m), which produce pixels with long lists. Rows are shuffled."""
    rng = np.random.default_rng(seed)
    n_dense = int(round(n * dense_frac))
    n_wide = n - n_dense
    wide = _cluster_means(rng, n_wide, 64, box, 0.5, 3.0, True)
    dense = _cluster_means(rng, n_dense, 8, box, 0.1, 0.4, False)
    means = np.concatenate([wide, dense], axis=0)
    perm = rng.permutation(n)
    means = means[perm]
    log_scales = rng.normal(-4.0, 1.0, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(0.0, 2.0, size=(n,))
    sh = _sh_coeffs(rng, n, sh_degree)
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), sh, sh_degree)


def camera_pinhole(position, target, width, height, fov_y_deg, near=0.2) -> Camera:
    """Look-at pinhole camera with square pixels and the principal point at the
    image centre; world up is -y."""
    c = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f = f / np.linalg.norm(f)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, f)
    if np.linalg.norm(right) < 1e-12:  # looking straight along the up axis
        right = np.array([1.0, 0.0, 0.0])
    right = right / np.linalg.norm(right)
    ydown = np.cross(f, right)
    r = np.stack([right, ydown, f], axis=0)
    t = -r @ c
    w2c = np.concatenate([r, t[:, None]], axis=1)
    fy = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return Camera(w2c, fy, fy, width / 2.0, height / 2.0, int(width), int(height), near)


def camera_orbit(radius, elevation_deg, azimuth_deg, width, height, fov_y_deg=60.0,
                 target=(0.0, 0.0, 0.0), near=0.2) -> Camera:
    el = math.radians(elevation_deg)
    az = math.radians(azimuth_deg)
    pos = np.array([radius * math.cos(el) * math.sin(az),
                    -radius * math.sin(el),
                    -radius * math.cos(el) * math.cos(az)]) + np.asarray(target, dtype=np.float64)
    return camera_pinhole(pos, target, width, height, fov_y_deg, near)


def camera_small(width: int = 128, height: int = 128) -> Camera:
    """Camera at (0, 0, -4) looking along +z with a 60 degree field of view."""
    return camera_pinhole((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), width, height, 60.0)


def camera_1080p(azimuth_deg: float = 0.0) -> Camera:
    return camera_orbit(30.0, 20.0, azimuth_deg, 1920, 1080, 60.0)


def cameras_sweep(n_poses: int = 32, width: int = 1600, height: int = 1040):
    return [camera_orbit(30.0, 20.0, 360.0 * k / n_poses, width, height, 60.0)
            for k in range(n_poses)]


def save_scene(path, scene: Scene) -> None:
    np.savez(path, means=scene.means, log_scales=scene.log_scales, quats=scene.quats,
             opacity_logits=scene.opacity_logits, sh=scene.sh,
             sh_degree=np.int64(scene.sh_degree))


def load_scene(path) -> Scene:
    z = np.load(path, allow_pickle=False)
    return Scene(z["means"], z["log_scales"], z["quats"], z["opacity_logits"], z["sh"],
                 int(z["sh_degree"]))
