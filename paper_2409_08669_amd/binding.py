"""ctypes binding of ``libadr.so`` (include/adr.h), names as in the C ABI.

Argument marshalling only: every stage of a frame runs in the HIP library.
PyTorch supplies device memory and the current stream. Importing this module
does not touch the GPU; loading the library fails loudly if it is not built.
"""
from __future__ import annotations

import ctypes
import math
import dataclasses
import pathlib

import numpy as np

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libadr.so"
_lib = None

ADR_OK = 0
ADR_E_INVALID = -1
ADR_E_OOM = -2
ADR_E_HIP = -3
ADR_E_UNSUPPORTED = -4
ADR_E_WORKSPACE = -5

ADR_CULL_3SIGMA = 0
ADR_CULL_ADAPTIVE = 1
ADR_CULL_AABB = 2

ADR_FLAG_TIMING = 1
ADR_FLAG_NO_EXACT_BAND = 2
ADR_FLAG_NO_QUAD_CULL = 4

STAGES = ("preprocess", "host_wait", "depth_sort", "inclusive_sum", "duplicate", "tile_sort", "ranges",
          "tile_order", "render", "load_sums")

EXPORTS = (
    "adr_create_scene", "adr_destroy_scene", "adr_scene_size", "adr_scene_bytes",
    "adr_workspace_create", "adr_workspace_destroy", "adr_render", "adr_render_backward", "adr_render_backward_load",
    "adr_workspace_stage_times", "adr_workspace_counters", "adr_last_error", "adr_version",
    "adr_server_create", "adr_server_destroy", "adr_server_submit", "adr_server_wait", "adr_clock_s",
)


class AdrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"adr status {status}: {msg}")
        self.status = status


class adr_scene_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("pointers_on_device", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class adr_camera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_double * 12), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("near_z", ctypes.c_double)]


class adr_render_params(ctypes.Structure):
    _fields_ = [("cull", ctypes.c_int32), ("lb_cap", ctypes.c_int32), ("alpha_low", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double), ("lowpass", ctypes.c_double),
                ("ewa_clamp", ctypes.c_double), ("background", ctypes.c_float * 3), ("flags", ctypes.c_uint32)]


class adr_frame(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("final_t", ctypes.c_void_p), ("l_iter", ctypes.c_void_p),
                ("l_blend", ctypes.c_void_p), ("load_sums", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p),
                ("keys", ctypes.c_void_p), ("values", ctypes.c_void_p), ("ranges", ctypes.c_void_p),
                ("pair_capacity", ctypes.c_int64), ("n_pairs", ctypes.c_int64)]


class adr_scene_grads(ctypes.Structure):
    _fields_ = [("d_means", ctypes.c_void_p), ("d_log_scales", ctypes.c_void_p), ("d_quats", ctypes.c_void_p),
                ("d_opacity_logits", ctypes.c_void_p), ("d_sh", ctypes.c_void_p)]


def lib_path() -> pathlib.Path:
    return _LIB_PATH


def load(path=None):
    """Loads the HIP library once; raises if it is missing (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    p = pathlib.Path(path) if path else _LIB_PATH
    if not p.exists():
        raise ImportError(f"{p} is not built; run `python -m paper_2409_08669_amd.build` (needs hipcc)")
    lib = ctypes.CDLL(str(p))
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.adr_create_scene.argtypes = [ctypes.POINTER(adr_scene_desc), ctypes.POINTER(vp)]
    lib.adr_create_scene.restype = i32
    lib.adr_destroy_scene.argtypes = [vp]
    lib.adr_destroy_scene.restype = None
    lib.adr_scene_size.argtypes = [vp]
    lib.adr_scene_size.restype = i64
    lib.adr_scene_bytes.argtypes = [vp]
    lib.adr_scene_bytes.restype = i64
    lib.adr_workspace_create.argtypes = [ctypes.POINTER(vp)]
    lib.adr_workspace_create.restype = i32
    lib.adr_workspace_destroy.argtypes = [vp]
    lib.adr_workspace_destroy.restype = None
    lib.adr_render.argtypes = [vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                               ctypes.POINTER(adr_frame), vp, vp]
    lib.adr_render.restype = i32
    lib.adr_render_backward.argtypes = [vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                                        ctypes.POINTER(adr_frame), vp, ctypes.POINTER(adr_scene_grads), vp, vp]
    lib.adr_render_backward.restype = i32
    lib.adr_render_backward_load.argtypes = [vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                                             ctypes.POINTER(adr_frame), vp, vp, ctypes.POINTER(adr_scene_grads), vp,
                                             vp]
    lib.adr_render_backward_load.restype = i32
    lib.adr_workspace_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    lib.adr_workspace_stage_times.restype = i32
    lib.adr_workspace_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), i32]
    lib.adr_workspace_counters.restype = i32
    lib.adr_server_create.argtypes = [i32, ctypes.POINTER(vp)]
    lib.adr_server_create.restype = i32
    lib.adr_server_destroy.argtypes = [vp]
    lib.adr_server_destroy.restype = None
    lib.adr_server_submit.argtypes = [vp, vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                                      ctypes.POINTER(adr_frame), ctypes.POINTER(ctypes.c_uint64)]
    lib.adr_server_submit.restype = i32
    lib.adr_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(adr_request_info)]
    lib.adr_server_wait.restype = i32
    lib.adr_clock_s.argtypes = []
    lib.adr_clock_s.restype = ctypes.c_double
    lib.adr_last_error.argtypes = []
    lib.adr_last_error.restype = ctypes.c_char_p
    lib.adr_version.argtypes = []
    lib.adr_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class adr_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


def last_error() -> str:
    return load().adr_last_error().decode()


def _check(status: int):
    if status != ADR_OK:
        raise AdrError(status, last_error())


@dataclasses.dataclass
class RenderParams:
    cull: int = ADR_CULL_AABB
    lb_cap: int = 0
    alpha_low: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    lowpass: float = 0.3
    ewa_clamp: float = 1.3
    background: tuple = (0.0, 0.0, 0.0)
    flags: int = 0

    def to_c(self) -> adr_render_params:
        p = adr_render_params()
        p.cull, p.lb_cap = int(self.cull), int(self.lb_cap)
        p.alpha_low, p.alpha_max, p.t_min = float(self.alpha_low), float(self.alpha_max), float(self.t_min)
        p.lowpass, p.ewa_clamp = float(self.lowpass), float(self.ewa_clamp)
        for i in range(3):
            p.background[i] = float(self.background[i])
        p.flags = int(self.flags)
        return p


def camera_to_c(cam) -> adr_camera:
    """Any object with world_to_cam (3x4), fx, fy, cx, cy, width, height, near."""
    c = adr_camera()
    w2c = np.asarray(cam.world_to_cam, dtype=np.float64).reshape(12)
    for i in range(12):
        c.world_to_cam[i] = float(w2c[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_z = float(getattr(cam, "near", 0.2))
    return c


class Scene:
    """Device copy of a Gaussian scene (adr_create_scene). Accepts numpy arrays
    (host) or torch tensors on the GPU; float32, row-major."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree: int):
        lib = load()
        arrays = [means, log_scales, quats, opacity_logits, sh]
        on_device = hasattr(means, "is_cuda") and bool(means.is_cuda)
        keep = []
        ptrs = []
        for a in arrays:
            if on_device:
                a = a.contiguous().float()
                keep.append(a)
                ptrs.append(a.data_ptr())
            else:
                a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
                keep.append(a)
                ptrs.append(a.ctypes.data)
        d = adr_scene_desc()
        d.n = int(keep[0].shape[0])
        d.sh_degree = int(sh_degree)
        d.pointers_on_device = 1 if on_device else 0
        d.means, d.log_scales, d.quats, d.opacity_logits, d.sh = ptrs
        h = ctypes.c_void_p()
        _check(lib.adr_create_scene(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.n = d.n
        self.sh_degree = int(sh_degree)

    @classmethod
    def from_synth(cls, s) -> "Scene":
        return cls(s.means, s.log_scales, s.quats, s.opacity_logits, s.sh, s.sh_degree)

    @property
    def handle(self):
        return self._h

    @property
    def bytes(self) -> int:
        return int(load().adr_scene_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().adr_destroy_scene(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """adr_workspace: per-stream scratch that grows on demand."""

    def __init__(self):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.adr_workspace_create(ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def stage_times(self) -> dict:
        buf = (ctypes.c_float * len(STAGES))()
        k = load().adr_workspace_stage_times(self._h, buf, len(STAGES))
        return {STAGES[i]: float(buf[i]) for i in range(k)}

    def counters(self) -> dict:
        buf = (ctypes.c_int64 * 6)()
        k = load().adr_workspace_counters(self._h, buf, 6)
        names = ("pairs", "visible", "band_redecisions", "t_replays", "depth_sort_bits", "bad_sort_indices")
        return {names[i]: int(buf[i]) for i in range(k)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().adr_workspace_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    return 0 if t is None else int(t.data_ptr())


def render(scene: Scene, cam, params: RenderParams, ws: Workspace, image, final_t=None, l_iter=None,
           l_blend=None, load_sums=None, tiles_touched=None, keys=None, values=None, ranges=None,
           pair_capacity: int = 0, stream=None) -> int:
    """adr_render into caller-allocated device tensors; returns the pair count.
    Raises AdrError on any non-OK status (ADR_E_WORKSPACE carries n_pairs)."""
    import torch

    lib = load()
    f = adr_frame()
    f.image, f.final_t, f.l_iter, f.l_blend = _ptr(image), _ptr(final_t), _ptr(l_iter), _ptr(l_blend)
    f.load_sums, f.tiles_touched = _ptr(load_sums), _ptr(tiles_touched)
    f.keys, f.values, f.ranges = _ptr(keys), _ptr(values), _ptr(ranges)
    f.pair_capacity = int(pair_capacity)
    c = camera_to_c(cam)
    p = params.to_c()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib.adr_render(scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f), ws.handle,
                        ctypes.c_void_p(int(stream)))
    if st == ADR_E_WORKSPACE:
        e = AdrError(st, last_error())
        e.n_pairs = int(f.n_pairs)
        raise e
    _check(st)
    return int(f.n_pairs)


def render_frame(scene: Scene, cam, params: RenderParams, ws: Workspace = None, debug: bool = False,
                 device: str = "cuda") -> dict:
    """Allocates the outputs with torch and renders one frame. With debug=True
    the per-Gaussian counts, sorted pairs and tile ranges are returned too
    (a first call sizes the pair buffers)."""
    import torch

    ws = ws or Workspace()
    w, h = int(cam.width), int(cam.height)
    tiles = ((w + 15) // 16) * ((h + 15) // 16)
    out = dict(
        image=torch.empty((3, h, w), dtype=torch.float32, device=device),
        final_t=torch.empty((h, w), dtype=torch.float32, device=device),
        l_iter=torch.empty((h, w), dtype=torch.int32, device=device),
        l_blend=torch.empty((h, w), dtype=torch.int32, device=device),
        load_sums=torch.zeros(4, dtype=torch.int64, device=device),
    )
    extra = {}
    cap = 0
    if debug:
        extra = dict(tiles_touched=torch.empty(max(scene.n, 1), dtype=torch.int32, device=device),
                     ranges=torch.empty((tiles, 2), dtype=torch.int32, device=device))
        n_pairs = render(scene, cam, params, ws, **out, **extra)
        cap = max(n_pairs, 1)
        extra["keys"] = torch.empty(cap, dtype=torch.int64, device=device)
        extra["values"] = torch.empty(cap, dtype=torch.int32, device=device)
    n_pairs = render(scene, cam, params, ws, **out, **extra, pair_capacity=cap)
    out.update(extra)
    out["n_pairs"] = n_pairs
    if debug:
        out["keys"] = out["keys"][:n_pairs]
        out["values"] = out["values"][:n_pairs]
        out["tiles_touched"] = out["tiles_touched"][:scene.n]
    out["workspace"] = ws
    return out


def render_backward(scene: Scene, cam, params: RenderParams, ws: Workspace, frame: dict, dl_dimage,
                    stream=None, dl_dload=None) -> dict:
    """adr_render_backward: gradients of L = sum(dl_dimage * image) with
    respect to the scene inputs, for the frame that the last render() on ws
    drew from the same scene, camera and params (frame: its outputs; final_t
    and l_iter are required). Returns float32 device tensors shaped like the
    scene arrays: means (N, 3), log_scales (N, 3), quats (N, 4),
    opacity_logits (N,), sh (N, K, 3). dl_dload (H, W), optional: dL/d(per-pixel
    load l_blend), taken through the alpha of every blended entry with slope 1
    (adr_render_backward_load)."""
    import torch

    lib = load()
    n, k = scene.n, (scene.sh_degree + 1) ** 2
    dev = frame["image"].device
    grads = dict(means=torch.empty((n, 3), device=dev), log_scales=torch.empty((n, 3), device=dev),
                 quats=torch.empty((n, 4), device=dev), opacity_logits=torch.empty((n,), device=dev),
                 sh=torch.empty((n, k, 3), device=dev))
    dl = dl_dimage.contiguous().float()
    f = adr_frame()
    f.image, f.final_t, f.l_iter = _ptr(frame["image"]), _ptr(frame.get("final_t")), _ptr(frame.get("l_iter"))
    g = adr_scene_grads()
    g.d_means, g.d_log_scales, g.d_quats = _ptr(grads["means"]), _ptr(grads["log_scales"]), _ptr(grads["quats"])
    g.d_opacity_logits, g.d_sh = _ptr(grads["opacity_logits"]), _ptr(grads["sh"])
    c = camera_to_c(cam)
    p = params.to_c()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    if dl_dload is None:
        _check(lib.adr_render_backward(scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f),
                                       ctypes.c_void_p(dl.data_ptr()), ctypes.byref(g), ws.handle,
                                       ctypes.c_void_p(int(stream))))
    else:
        dload = dl_dload.contiguous().float()
        _check(lib.adr_render_backward_load(scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f),
                                            ctypes.c_void_p(dl.data_ptr()), ctypes.c_void_p(dload.data_ptr()),
                                            ctypes.byref(g), ws.handle, ctypes.c_void_p(int(stream))))
    return grads


def _autograd_function():
    import torch

    class RenderFn(torch.autograd.Function):
        """image = render(scene inputs); backward through adr_render_backward."""

        @staticmethod
        def forward(ctx, means, log_scales, quats, opacity_logits, sh, cam, params, ws):
            scene = Scene(means.detach(), log_scales.detach(), quats.detach(), opacity_logits.detach(),
                          sh.detach(), int(round(math.sqrt(sh.shape[1]))) - 1)
            h, w = int(cam.height), int(cam.width)
            dev = means.device
            frame = dict(image=torch.empty((3, h, w), device=dev), final_t=torch.empty((h, w), device=dev),
                         l_iter=torch.empty((h, w), dtype=torch.int32, device=dev))
            render(scene, cam, params, ws, **frame)
            ctx.state = (scene, cam, params, ws, frame)
            return frame["image"].clone()

        @staticmethod
        def backward(ctx, grad_image):
            scene, cam, params, ws, frame = ctx.state
            g = render_backward(scene, cam, params, ws, frame, grad_image)
            return g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None, None, None

    return RenderFn


def render_differentiable(means, log_scales, quats, opacity_logits, sh, cam, params: RenderParams,
                          ws: Workspace = None):
    """The image as a differentiable function of the scene inputs (torch
    tensors on the GPU; sh of shape (N, K, 3)). The backward pass must run
    before ws renders another frame."""
    global _render_fn
    if _render_fn is None:
        _render_fn = _autograd_function()
    return _render_fn.apply(means, log_scales, quats, opacity_logits, sh, cam, params, ws or Workspace())


_render_fn = None


def load_stats_from_sums(sums, n_pixels: int):
    """Exact (mean, population std) from the integer sums (sum, sum of squares)
    that adr_render writes; Eq. 13 over all H x W pixels."""
    import math
    s1, s2 = int(sums[0]), int(sums[1])
    mean = s1 / n_pixels
    var = (n_pixels * s2 - s1 * s1) / (n_pixels * n_pixels)
    return mean, math.sqrt(max(var, 0.0))


def clock_s() -> float:
    """The steady clock the server time-stamps requests with (seconds)."""
    return float(load().adr_clock_s())


class Server:
    """adr_server: n_slots render slots (host thread + HIP stream + workspace
    each) consuming queued frame requests over resident scenes."""

    def __init__(self, n_slots: int = 4):
        h = ctypes.c_void_p()
        _check(load().adr_server_create(int(n_slots), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> objects that must outlive the request

    def submit(self, scene: Scene, cam, params: RenderParams, image, final_t=None, l_iter=None, l_blend=None,
               load_sums=None) -> int:
        """Queues one frame into caller-allocated device tensors; returns its
        ticket. The tensors and the scene must stay alive until wait()."""
        f = adr_frame()
        f.image, f.final_t, f.l_iter, f.l_blend = _ptr(image), _ptr(final_t), _ptr(l_iter), _ptr(l_blend)
        f.load_sums = _ptr(load_sums)
        c, p = camera_to_c(cam), params.to_c()
        t = ctypes.c_uint64()
        _check(load().adr_server_submit(self._h, scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f),
                                        ctypes.byref(t)))
        self._keep[int(t.value)] = (scene, image, final_t, l_iter, l_blend, load_sums)
        return int(t.value)

    def wait(self, ticket: int) -> dict:
        """Blocks until the frame is done; returns its status, pair count and
        time stamps (submit, start, done; seconds of clock_s())."""
        info = adr_request_info()
        _check(load().adr_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(info)))
        self._keep.pop(int(ticket), None)
        out = dict(status=int(info.status), n_pairs=int(info.n_pairs), submit_s=info.submit_s,
                   start_s=info.start_s, done_s=info.done_s)
        if info.status != ADR_OK:
            raise AdrError(int(info.status), last_error())
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().adr_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
