"""The C-ABI library loads on the host, exports every symbol the header
declares, and rejects bad arguments before anything reaches a GPU. CPU only:
none of these calls enqueues work."""
import ctypes
import pathlib
import re

import numpy as np
import pytest

from synth import camera_small

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "adr.h"


def _lib():
    from paper_2409_08669_amd import binding
    if not binding.lib_path().exists():
        pytest.skip("libadr.so not built (run python -m paper_2409_08669_amd.build)")
    return binding, binding.load()


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("adr_create_scene", "adr_render", "adr_render_backward", "adr_destroy_scene",
                     "adr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    binding, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(binding.EXPORTS) == set(declared_functions())


def test_version_string():
    _, lib = _lib()
    assert lib.adr_version().startswith(b"adr-gfx950")


def test_create_scene_rejects_bad_arguments_on_host():
    binding, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.adr_create_scene(None, None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "NULL" in binding.last_error()
    d = binding.adr_scene_desc()
    d.n, d.sh_degree = 10, 4
    assert lib.adr_create_scene(ctypes.byref(d), None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "sh_degree" in binding.last_error()
    d.sh_degree, d.n = 0, -1
    assert lib.adr_create_scene(ctypes.byref(d), None, ctypes.byref(h)) == binding.ADR_E_INVALID
    d.n = 5  # NULL arrays with n > 0
    assert lib.adr_create_scene(ctypes.byref(d), None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert h.value is None


def _fake_desc(binding, n=5, on_device=1, borrow=1, quats=4096):
    d = binding.adr_scene_desc()
    d.n, d.sh_degree, d.pointers_on_device, d.borrow = n, 0, on_device, borrow
    d.means, d.log_scales, d.opacity_logits, d.sh = 1024, 2048, 3072, 5120  # never dereferenced
    d.quats = quats
    return d


def test_borrowed_scene_needs_aligned_device_pointers():
    """borrow = 1 keeps the caller's arrays: host pointers, or quaternions not
    16-byte aligned (read as one 16-byte load), are rejected before any device
    call."""
    binding, lib = _lib()
    h = ctypes.c_void_p()
    d = _fake_desc(binding, on_device=0)
    assert lib.adr_create_scene(ctypes.byref(d), None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "device pointers" in binding.last_error()
    d = _fake_desc(binding, quats=4100)
    assert lib.adr_create_scene(ctypes.byref(d), None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "aligned" in binding.last_error()
    assert h.value is None


def test_allocator_needs_both_functions():
    """A caller allocator with alloc but no free (or the reverse) is refused
    by the scene and the workspace before anything is allocated."""
    binding, lib = _lib()
    calls = []

    def _alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    a = binding.adr_allocator()
    a.alloc = binding.ALLOC_FN(_alloc)  # free left NULL
    h = ctypes.c_void_p()
    assert lib.adr_workspace_create(ctypes.byref(a), ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "alloc and free" in binding.last_error()
    d = _fake_desc(binding, borrow=0)
    assert lib.adr_create_scene(ctypes.byref(d), ctypes.byref(a), ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "alloc and free" in binding.last_error()
    assert calls == [] and h.value is None


def test_workspace_bytes_follow_the_arena_layout():
    """adr_workspace_bytes is host arithmetic: per Gaussian the 64-byte render
    record, the 32-byte FP64 record, the 8-byte tile rectangle, three u32
    arrays and the double-buffered depth keys and ids (16 bytes), plus
    per-block scan, Preprocess and radix partials; per pair the
    double-buffered tile ids and Gaussian ids (16 bytes); per tile the ranges
    (8), the render order (4) and the load partials of four waves (128),
    plus the tile order's bucket counts (33 words per 16 x 16 superblock,
    sized for the most superblocks a grid of that many tiles can have)."""
    _, lib = _lib()
    base = lib.adr_workspace_bytes(0, 0, 0)
    assert base > 0 and base % 256 == 0
    n, p, t = 1_000_000, 4_000_000, 8160
    dg = lib.adr_workspace_bytes(n, 0, 0) - base
    dp = lib.adr_workspace_bytes(0, p, 0) - base
    dt = lib.adr_workspace_bytes(0, 0, t) - base
    assert 132 * n <= dg <= 132.7 * n  # + radix counts, scan and Preprocess partials
    assert 16 * p <= dp <= 16.3 * p  # + radix counts and chunk starts
    order_counts = 33 * 4 * (t // 256 + t // 16 + 2)
    assert 140 * t + order_counts - 1024 <= dt <= 140 * t + order_counts + 4096  # base holds the t = 0 share
    assert lib.adr_workspace_bytes(n, p, t) == base + dg + dp + dt
    assert lib.adr_workspace_bytes(-1, 0, 0) == -1


def test_workspace_reserve_and_capacity_reject_bad_arguments():
    binding, lib = _lib()
    assert lib.adr_workspace_reserve(None, 1, 1, 1) == binding.ADR_E_INVALID
    assert lib.adr_workspace_capacity_bytes(None) == -1


def test_render_rejects_bad_arguments_on_host():
    binding, lib = _lib()
    cam = binding.adr_camera()
    cam.fx = cam.fy = 100.0
    cam.width = cam.height = 64
    cam.cx = cam.cy = 32.0
    cam.near_z = 0.2
    p = binding.RenderParams().to_c()
    f = binding.adr_frame()
    # NULL scene
    assert lib.adr_render(None, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), None, None) == \
        binding.ADR_E_INVALID
    fake = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    # missing image
    assert lib.adr_render(fake, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), fake, None) == \
        binding.ADR_E_INVALID
    assert "image" in binding.last_error()
    f.image = 1
    for field, value in (("width", 0), ("height", 70000)):
        c2 = binding.adr_camera.from_buffer_copy(cam)
        setattr(c2, field, value)
        assert lib.adr_render(fake, ctypes.byref(c2), ctypes.byref(p), ctypes.byref(f), fake, None) == \
            binding.ADR_E_INVALID
    for field, value in (("cull", 7), ("alpha_low", 0.0), ("alpha_low", 0.995), ("t_min", 0.0), ("lb_cap", -1),
                         ("lowpass", -1.0), ("ewa_clamp", 0.0)):
        p2 = binding.RenderParams().to_c()
        setattr(p2, field, value)
        assert lib.adr_render(fake, ctypes.byref(cam), ctypes.byref(p2), ctypes.byref(f), fake, None) == \
            binding.ADR_E_INVALID, field
    c3 = binding.adr_camera.from_buffer_copy(cam)
    c3.world_to_cam[0] = float("nan")
    assert lib.adr_render(fake, ctypes.byref(c3), ctypes.byref(p), ctypes.byref(f), fake, None) == \
        binding.ADR_E_INVALID


def test_noalloc_render_rejects_bad_arguments_on_host():
    """adr_render_noalloc validates like adr_render before it looks up its
    device scratch: NULL handles, a missing image, bad camera and params."""
    binding, lib = _lib()
    assert lib.adr_noalloc_scratch_bytes() == 256 << 20
    cam = binding.adr_camera()
    cam.fx = cam.fy = 100.0
    cam.width = cam.height = 64
    cam.cx = cam.cy = 32.0
    cam.near_z = 0.2
    p = binding.RenderParams().to_c()
    f = binding.adr_frame()
    assert lib.adr_render_noalloc(None, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), None) == \
        binding.ADR_E_INVALID
    fake = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    assert lib.adr_render_noalloc(fake, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), None) == \
        binding.ADR_E_INVALID
    assert "image" in binding.last_error()
    f.image = 1
    c2 = binding.adr_camera.from_buffer_copy(cam)
    c2.width = 0
    assert lib.adr_render_noalloc(fake, ctypes.byref(c2), ctypes.byref(p), ctypes.byref(f), None) == \
        binding.ADR_E_INVALID
    p2 = binding.RenderParams().to_c()
    p2.alpha_low = 0.0
    assert lib.adr_render_noalloc(fake, ctypes.byref(cam), ctypes.byref(p2), ctypes.byref(f), None) == \
        binding.ADR_E_INVALID


def test_backward_rejects_missing_arguments_on_the_host():
    """adr_render_backward checks its arguments before touching the device:
    NULL handles, and a forward frame without final_t or l_iter."""
    binding, lib = _lib()
    assert lib.adr_render_backward(None, None, None, None, None, None, None, None) == binding.ADR_E_INVALID
    fake = ctypes.c_void_p(1)
    cam = binding.camera_to_c(camera_small(32, 32))
    p = binding.RenderParams().to_c()
    f = binding.adr_frame()
    f.image = 1  # a forward frame with an image but neither final_t nor l_iter
    g = binding.adr_scene_grads()
    assert lib.adr_render_backward(fake, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), fake,
                                   ctypes.byref(g), fake, None) == binding.ADR_E_INVALID
    assert "final_t and l_iter" in binding.last_error()


def test_stage_times_and_counters_without_frames():
    _, lib = _lib()
    buf = (ctypes.c_float * 7)()
    assert lib.adr_workspace_stage_times(None, buf, 7) == 0
    cbuf = (ctypes.c_int64 * 6)()
    assert lib.adr_workspace_counters(None, cbuf, 6) == 0


def test_missing_library_fails_loudly(tmp_path):
    from paper_2409_08669_amd import binding
    saved = binding._lib
    try:
        binding._lib = None
        with pytest.raises(ImportError):
            binding.load(tmp_path / "nope.so")
    finally:
        binding._lib = saved


def test_package_does_not_import_the_oracle():
    pkg = ROOT / "paper_2409_08669_amd"
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + list(pkg.rglob("*.h")):
        text = f.read_text()
        assert "import oracle" not in text and "from oracle" not in text, f
        assert "adr_oracle" not in text, f


def test_server_rejects_bad_arguments_on_host():
    """Serving entry points validate on the host before touching a device."""
    binding, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.adr_server_create(None, ctypes.byref(h)) == binding.ADR_E_INVALID
    for slots, batch, budget in ((0, 4, 1 << 30), (65, 4, 1 << 30), (4, 0, 1 << 30), (4, 65, 1 << 30), (4, 4, 0)):
        cfg = binding.adr_server_config()
        cfg.n_slots, cfg.max_batch, cfg.memory_budget = slots, batch, budget
        assert lib.adr_server_create(ctypes.byref(cfg), ctypes.byref(h)) == binding.ADR_E_INVALID
    assert not h.value
    t = ctypes.c_uint64()
    cam = binding.adr_camera()
    p = binding.RenderParams().to_c()
    f = binding.adr_frame()
    assert lib.adr_server_submit(None, None, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), 0.0,
                                 ctypes.byref(t)) == binding.ADR_E_INVALID
    fake = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    assert lib.adr_server_submit(fake, fake, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f), 0.0,
                                 ctypes.byref(t)) == binding.ADR_E_INVALID  # no image, zero-size camera
    assert lib.adr_server_wait(None, 1, None) == binding.ADR_E_INVALID
    assert lib.adr_server_stats_get(None, None) == binding.ADR_E_INVALID
    assert lib.adr_clock_s() > 0.0
