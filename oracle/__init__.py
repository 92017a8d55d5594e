"""Plain FP64 CPU oracle for the AdR-Gaussian forward rasterizer.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import it: only the
tests, the smoke check of the entry module and the CPU-baseline leg of the
benchmark use it. It shares no code with the HIP library.
"""
from .adr_oracle import (  # noqa: F401
    Params,
    CULL_3SIGMA,
    CULL_ADAPTIVE,
    CULL_AABB,
    quat_to_rotmat,
    covariance_3d,
    cull_radii,
    n_tiles,
    sh_basis,
    camera_position,
    sh_to_rgb,
    preprocess,
    tile_rects,
    duplicate_and_sort,
    tile_ranges,
    render_pixels,
    render_image,
    render_frame,
    load_stats,
    psnr,
    brute_force_render,
)
