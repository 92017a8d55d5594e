"""A hand-placed scene in which some pixels stop (T < t_min) while the rest of
their 8 x 8 quadrant keeps blending, and the entry right after the stop is a
Gaussian whose FP32 exponent has no usable error bound (a needle with a
projected axis ratio above 2000), so the blend decides it in FP64 only.
Gaussian 0 is a broad faint Gaussian behind everything that reaches the
stopped pixels.

Such a stopped pixel must keep its state: it blends nothing after the entry
that stopped it (Eq. 3 ends the blend there), whatever the next entry is.

Layout (camera_small(32, 32): camera at z = -4 looking along +z):
* Gaussian 0: centre at pixel (16, 16), depth 7, sigma 3 world units,
  opacity 0.5;
* n_weak weak walls (opacity ~0.3) and then three strong walls (opacity
  ~0.982, below alpha_max so that no transmittance ties t_min) at pixel
  (1.5, 1.5), depths 2.8 ... 3.0, 6 px sigma: the pixels closest to
  (1.5, 1.5) stop at the last wall, entry 3 + n_weak of the tile's list;
* the needle: centre at pixel (1.5, 1.5), depth 4.5, scales (500, 1e-4,
  1e-4) world units along (x, y, z).
"""
import math

import numpy as np

from synth import Scene, camera_small

_Y00 = 0.28209479177387814  # degree-0 SH basis value: colour = 0.5 + _Y00 * sh


def stop_scene(n_weak: int = 0):
    cam = camera_small(32, 32)

    def world_at(px, py, z_cam):
        return [(px + 0.5 - cam.cx) * z_cam / cam.fx, (py + 0.5 - cam.cy) * z_cam / cam.fy, z_cam - 4.0]

    means, log_scales, quats, logits, rgb = [], [], [], [], []

    def add(mean, scales, logit, colour):
        means.append(mean)
        log_scales.append([math.log(v) for v in scales])
        quats.append([1.0, 0.0, 0.0, 0.0])
        logits.append(logit)
        rgb.append(colour)

    add(world_at(16, 16, 7.0), (3.0, 3.0, 3.0), 0.0, (0.2, 0.4, 0.6))
    walls = [-0.85] * n_weak + [4.0] * 3
    depths = np.linspace(2.8, 3.0, len(walls))
    for k, (lg, z) in enumerate(zip(walls, depths)):
        s = 6.0 * z / cam.fx
        add(world_at(1.5, 1.5, z), (s, s, s), lg, (0.9, 0.1 * k, 0.1))
    add(world_at(1.5, 1.5, 4.5), (500.0, 1e-4, 1e-4), 3.0, (0.1, 0.9, 0.2))
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    sh = ((np.asarray(rgb) - 0.5) / _Y00).reshape(-1, 1, 3)
    scene = Scene(f32(means), f32(log_scales), f32(quats), f32(logits), f32(sh), 0)
    return scene, cam, len(walls)
