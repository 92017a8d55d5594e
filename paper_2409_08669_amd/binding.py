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
    "adr_workspace_create", "adr_workspace_destroy", "adr_workspace_reserve", "adr_workspace_bytes",
    "adr_workspace_capacity_bytes", "adr_render", "adr_render_backward", "adr_render_backward_load",
    "adr_workspace_stage_times", "adr_workspace_counters", "adr_last_error", "adr_version",
    "adr_server_create", "adr_server_destroy", "adr_server_submit", "adr_server_wait", "adr_server_stats_get",
    "adr_clock_s", "adr_render_noalloc", "adr_noalloc_scratch_bytes",
)


class AdrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"adr status {status}: {msg}")
        self.status = status


class adr_scene_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("pointers_on_device", ctypes.c_int32),
                ("borrow", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity_logits", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class adr_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


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
                ("l_blend", ctypes.c_void_p), ("load_sums", ctypes.c_void_p), ("load_stats", ctypes.c_void_p),
                ("tiles_touched", ctypes.c_void_p),
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
    lib.adr_create_scene.argtypes = [ctypes.POINTER(adr_scene_desc), ctypes.POINTER(adr_allocator),
                                     ctypes.POINTER(vp)]
    lib.adr_create_scene.restype = i32
    lib.adr_destroy_scene.argtypes = [vp]
    lib.adr_destroy_scene.restype = None
    lib.adr_scene_size.argtypes = [vp]
    lib.adr_scene_size.restype = i64
    lib.adr_scene_bytes.argtypes = [vp]
    lib.adr_scene_bytes.restype = i64
    lib.adr_workspace_create.argtypes = [ctypes.POINTER(adr_allocator), ctypes.POINTER(vp)]
    lib.adr_workspace_create.restype = i32
    lib.adr_workspace_destroy.argtypes = [vp]
    lib.adr_workspace_destroy.restype = None
    lib.adr_workspace_reserve.argtypes = [vp, i64, i64, i64]
    lib.adr_workspace_reserve.restype = i32
    lib.adr_workspace_bytes.argtypes = [i64, i64, i64]
    lib.adr_workspace_bytes.restype = i64
    lib.adr_workspace_capacity_bytes.argtypes = [vp]
    lib.adr_workspace_capacity_bytes.restype = i64
    lib.adr_render.argtypes = [vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                               ctypes.POINTER(adr_frame), vp, vp]
    lib.adr_render.restype = i32
    lib.adr_render_noalloc.argtypes = [vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                                       ctypes.POINTER(adr_frame), vp]
    lib.adr_render_noalloc.restype = i32
    lib.adr_noalloc_scratch_bytes.argtypes = []
    lib.adr_noalloc_scratch_bytes.restype = i64
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
    lib.adr_server_create.argtypes = [ctypes.POINTER(adr_server_config), ctypes.POINTER(vp)]
    lib.adr_server_create.restype = i32
    lib.adr_server_destroy.argtypes = [vp]
    lib.adr_server_destroy.restype = None
    lib.adr_server_submit.argtypes = [vp, vp, ctypes.POINTER(adr_camera), ctypes.POINTER(adr_render_params),
                                      ctypes.POINTER(adr_frame), ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
    lib.adr_server_submit.restype = i32
    lib.adr_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(adr_request_info)]
    lib.adr_server_wait.restype = i32
    lib.adr_server_stats_get.argtypes = [vp, ctypes.POINTER(adr_server_stats)]
    lib.adr_server_stats_get.restype = i32
    lib.adr_clock_s.argtypes = []
    lib.adr_clock_s.restype = ctypes.c_double
    lib.adr_last_error.argtypes = []
    lib.adr_last_error.restype = ctypes.c_char_p
    lib.adr_version.argtypes = []
    lib.adr_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class adr_server_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("memory_budget", ctypes.c_int64)]


class adr_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("n_pairs", ctypes.c_int64),
                ("batch_id", ctypes.c_int64), ("footprint", ctypes.c_int64), ("arrival_s", ctypes.c_double),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class adr_server_stats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("batches", ctypes.c_int64), ("max_batch_seen", ctypes.c_int32),
                ("reserved1", ctypes.c_int32), ("reserved_bytes_peak", ctypes.c_int64),
                ("pool_bytes", ctypes.c_int64)]


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


def torch_allocator(device=None):
    """An adr_allocator backed by torch's caching allocator: alloc takes a
    block for the given stream, free hands it back (torch reuses it only for
    work ordered after the frame on that stream). Keep the returned object
    alive as long as anything allocated through it."""
    import torch

    dev = torch.cuda.current_device() if device is None else int(device)

    def _alloc(nbytes, stream, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0)))
        except Exception:  # reported to the library as a failed allocation (ADR_E_OOM)
            return None

    def _free(ptr, nbytes, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = adr_allocator()
    a.alloc, a.free, a.ctx = ALLOC_FN(_alloc), FREE_FN(_free), None
    return a


class Scene:
    """A Gaussian scene (adr_create_scene). Accepts numpy arrays (host) or
    torch tensors on the GPU; float32, row-major. borrow=True (GPU tensors
    only) keeps the caller's tensors and reads them in place; the scene holds
    references to them."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree: int, borrow: bool = False,
                 allocator=None):
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
        d.borrow = 1 if borrow else 0
        d.means, d.log_scales, d.quats, d.opacity_logits, d.sh = ptrs
        h = ctypes.c_void_p()
        self._allocator = allocator
        _check(lib.adr_create_scene(ctypes.byref(d), ctypes.byref(allocator) if allocator is not None else None,
                                    ctypes.byref(h)))
        self._h = h
        self._borrowed = keep if borrow else None  # the arrays a borrowed scene reads
        self.n = d.n
        self.sh_degree = int(sh_degree)

    @classmethod
    def from_synth(cls, s, **kw) -> "Scene":
        return cls(s.means, s.log_scales, s.quats, s.opacity_logits, s.sh, s.sh_degree, **kw)

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
            self._borrowed = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """adr_workspace: per-stream scratch that grows on demand. allocator:
    None (the library's hipMalloc arenas, kept until reserve() or close() when
    replaced), "torch" (torch's caching allocator) or an adr_allocator."""

    def __init__(self, allocator=None):
        lib = load()
        if allocator == "torch":
            allocator = torch_allocator()
        self._allocator = allocator
        h = ctypes.c_void_p()
        _check(lib.adr_workspace_create(ctypes.byref(allocator) if allocator is not None else None,
                                        ctypes.byref(h)))
        self._h = h

    def reserve(self, n_gauss: int, n_pairs: int, n_tiles: int):
        """adr_workspace_reserve: grow ahead of time (synchronises the device)."""
        _check(load().adr_workspace_reserve(self._h, int(n_gauss), int(n_pairs), int(n_tiles)))

    @property
    def capacity_bytes(self) -> int:
        return int(load().adr_workspace_capacity_bytes(self._h))

    @property
    def handle(self):
        return self._h

    def stage_times(self) -> dict:
        buf = (ctypes.c_float * len(STAGES))()
        k = load().adr_workspace_stage_times(self._h, buf, len(STAGES))
        return {STAGES[i]: float(buf[i]) for i in range(k)}

    @staticmethod
    def bytes_for(n_gauss: int, n_pairs: int, n_tiles: int) -> int:
        """adr_workspace_bytes: device bytes one frame slot needs (a workspace holds three)."""
        return int(load().adr_workspace_bytes(int(n_gauss), int(n_pairs), int(n_tiles)))

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


def _frame(image, final_t, l_iter, l_blend, load_sums, load_stats, tiles_touched, keys, values, ranges,
           pair_capacity) -> adr_frame:
    f = adr_frame()
    f.image, f.final_t, f.l_iter, f.l_blend = _ptr(image), _ptr(final_t), _ptr(l_iter), _ptr(l_blend)
    f.load_sums, f.load_stats, f.tiles_touched = _ptr(load_sums), _ptr(load_stats), _ptr(tiles_touched)
    f.keys, f.values, f.ranges = _ptr(keys), _ptr(values), _ptr(ranges)
    f.pair_capacity = int(pair_capacity)
    return f


def _finish(st: int, f: adr_frame) -> int:
    if st == ADR_E_WORKSPACE:
        e = AdrError(st, last_error())
        e.n_pairs = int(f.n_pairs)
        raise e
    _check(st)
    return int(f.n_pairs)


def render(scene: Scene, cam, params: RenderParams, ws: Workspace, image, final_t=None, l_iter=None,
           l_blend=None, load_sums=None, load_stats=None, tiles_touched=None, keys=None, values=None, ranges=None,
           pair_capacity: int = 0, stream=None) -> int:
    """adr_render into caller-allocated device tensors; returns the pair count.
    Raises AdrError on any non-OK status (ADR_E_WORKSPACE carries n_pairs)."""
    import torch

    lib = load()
    f = _frame(image, final_t, l_iter, l_blend, load_sums, load_stats, tiles_touched, keys, values, ranges,
               pair_capacity)
    c = camera_to_c(cam)
    p = params.to_c()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib.adr_render(scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f), ws.handle,
                        ctypes.c_void_p(int(stream)))
    return _finish(st, f)


def render_noalloc(scene: Scene, cam, params: RenderParams, image, final_t=None, l_iter=None, l_blend=None,
                   load_sums=None, load_stats=None, tiles_touched=None, keys=None, values=None, ranges=None,
                   pair_capacity: int = 0, stream=None) -> int:
    """adr_render_noalloc (no workspace; the library's fixed device scratch)
    into caller-allocated device tensors; returns the pair count. Raises
    AdrError on any non-OK status (ADR_E_WORKSPACE carries n_pairs)."""
    import torch

    lib = load()
    f = _frame(image, final_t, l_iter, l_blend, load_sums, load_stats, tiles_touched, keys, values, ranges,
               pair_capacity)
    c = camera_to_c(cam)
    p = params.to_c()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib.adr_render_noalloc(scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f),
                                ctypes.c_void_p(int(stream)))
    return _finish(st, f)


def noalloc_scratch_bytes() -> int:
    return int(load().adr_noalloc_scratch_bytes())


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
        load_stats=torch.zeros(4, dtype=torch.float64, device=device),
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
            # zero-copy: the scene reads the tensors in place until backward
            scene = Scene(means.detach(), log_scales.detach(), quats.detach(), opacity_logits.detach(),
                          sh.detach(), int(round(math.sqrt(sh.shape[1]))) - 1, borrow=True)
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


def clock_s() -> float:
    """The steady clock the server time-stamps requests with (seconds)."""
    return float(load().adr_clock_s())


class Server:
    """adr_server: continuous batching of render requests over resident
    scenes (n_slots requests in flight, blends of up to max_batch frames per
    launch, admission against memory_budget device bytes)."""

    def __init__(self, n_slots: int = 8, max_batch: int = 16, memory_budget: int = 16 << 30):
        cfg = adr_server_config()
        cfg.n_slots, cfg.max_batch, cfg.memory_budget = int(n_slots), int(max_batch), int(memory_budget)
        h = ctypes.c_void_p()
        _check(load().adr_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> objects that must outlive the request

    def submit(self, scene: Scene, cam, params: RenderParams, image, final_t=None, l_iter=None, l_blend=None,
               load_sums=None, load_stats=None, arrival_s: float = 0.0) -> int:
        """Queues one frame into caller-allocated device tensors; returns its
        ticket. arrival_s (clock_s() seconds; 0 = now) is the origin of its
        latency. The tensors and the scene must stay alive until wait()."""
        f = adr_frame()
        f.image, f.final_t, f.l_iter, f.l_blend = _ptr(image), _ptr(final_t), _ptr(l_iter), _ptr(l_blend)
        f.load_sums, f.load_stats = _ptr(load_sums), _ptr(load_stats)
        c, p = camera_to_c(cam), params.to_c()
        t = ctypes.c_uint64()
        _check(load().adr_server_submit(self._h, scene.handle, ctypes.byref(c), ctypes.byref(p), ctypes.byref(f),
                                        float(arrival_s), ctypes.byref(t)))
        self._keep[int(t.value)] = (scene, image, final_t, l_iter, l_blend, load_sums, load_stats)
        return int(t.value)

    def wait(self, ticket: int) -> dict:
        """Blocks until the frame is done; returns its status, pair count,
        batch, footprint and time stamps (clock_s() seconds)."""
        info = adr_request_info()
        _check(load().adr_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(info)))
        self._keep.pop(int(ticket), None)
        out = {k: getattr(info, k) for k, _ in adr_request_info._fields_}
        if info.status != ADR_OK:
            raise AdrError(int(info.status), last_error())
        return out

    def stats(self) -> dict:
        st = adr_server_stats()
        _check(load().adr_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in adr_server_stats._fields_ if not k.startswith("reserved1")}

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
