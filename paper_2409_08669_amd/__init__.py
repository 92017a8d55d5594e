"""MI355X (gfx950) AdR-Gaussian tile rasterizer.

The compute path is the HIP library ``libadr.so`` behind the C ABI declared in
``include/adr.h``; ``binding`` marshals arguments to it with ctypes. There is
no CPU fallback: calling into the binding without the built library raises.
"""
from .binding import (  # noqa: F401
    ADR_CULL_3SIGMA,
    ADR_CULL_ADAPTIVE,
    ADR_CULL_AABB,
    ADR_FLAG_TIMING,
    ADR_FLAG_NO_EXACT_BAND,
    ADR_FLAG_NO_QUAD_CULL,
    AdrError,
    RenderParams,
    Scene,
    Server,
    Workspace,
    clock_s,
    render_backward,
    render_differentiable,
    load,
    render,
    render_frame,
    render_noalloc,
    noalloc_scratch_bytes,
    torch_allocator,
)
