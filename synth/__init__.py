"""Seeded synthetic scenes and cameras shared by the oracle side and the HIP side.

This package only draws random inputs and builds camera matrices. It holds none
of the rasterizer's arithmetic (no projection, no covariance, no SH, no culling),
so that the oracle and the HIP path share nothing but their inputs.
"""
from .scenes import (  # noqa: F401
    Scene,
    Camera,
    scene_small,
    scene_small_sh3,
    scene_needles,
    scene_clusters,
    scene_heavy,
    camera_pinhole,
    camera_orbit,
    camera_small,
    camera_1080p,
    cameras_sweep,
    save_scene,
    load_scene,
)
