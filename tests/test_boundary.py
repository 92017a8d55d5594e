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
    assert lib.adr_create_scene(None, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "NULL" in binding.last_error()
    d = binding.adr_scene_desc()
    d.n, d.sh_degree = 10, 4
    assert lib.adr_create_scene(ctypes.byref(d), ctypes.byref(h)) == binding.ADR_E_INVALID
    assert "sh_degree" in binding.last_error()
    d.sh_degree, d.n = 0, -1
    assert lib.adr_create_scene(ctypes.byref(d), ctypes.byref(h)) == binding.ADR_E_INVALID
    d.n = 5  # NULL arrays with n > 0
    assert lib.adr_create_scene(ctypes.byref(d), ctypes.byref(h)) == binding.ADR_E_INVALID
    assert h.value is None


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
    cbuf = (ctypes.c_int64 * 5)()
    assert lib.adr_workspace_counters(None, cbuf, 5) == 0


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
    for n in (0, -1, 65):
        assert lib.adr_server_create(n, ctypes.byref(h)) == binding.ADR_E_INVALID
    assert lib.adr_server_create(4, None) == binding.ADR_E_INVALID
    t = ctypes.c_uint64()
    cam = binding.adr_camera()
    p = binding.RenderParams().to_c()
    f = binding.adr_frame()
    assert lib.adr_server_submit(None, None, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f),
                                 ctypes.byref(t)) == binding.ADR_E_INVALID
    fake = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    assert lib.adr_server_submit(fake, fake, ctypes.byref(cam), ctypes.byref(p), ctypes.byref(f),
                                 ctypes.byref(t)) == binding.ADR_E_INVALID  # no image, zero-size camera
    assert lib.adr_server_wait(None, 1, None) == binding.ADR_E_INVALID
    assert lib.adr_clock_s() > 0.0


def test_serving_is_switched_off_and_says_so():
    binding, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.adr_server_create(4, ctypes.byref(h)) == binding.ADR_E_UNSUPPORTED
    assert "switched off" in binding.last_error() and not h.value
