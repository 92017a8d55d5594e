"""Gradients through the C ABI (adr_render_backward) against the FP64
gradient oracle: every scene input (means, log-scales, quaternions, opacity
logits, SH degree 3) within 1e-3 of the largest oracle value of its array,
for each cull mode, and the same for every mode (the culling is lossless).
Runs on an MI355X only."""
import numpy as np
import pytest

import oracle as O
from oracle import adr_grad as G
from synth import scene_small_sh3, camera_small, camera_orbit, scene_small

pytestmark = pytest.mark.gpu

KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")
REL_TOL = 1e-3


def say(msg):
    print(f"[gpu-backward] {msg}", flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08669_amd as P
    P.load()
    return P


def f32(scene):
    """The scene with every input rounded to float32, the precision the
    library reads, so that both sides differentiate the same function."""
    from synth import Scene
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return Scene(r(scene.means), r(scene.log_scales), r(scene.quats), r(scene.opacity_logits), r(scene.sh),
                 scene.sh_degree)


def gpu_grads(P, scene, cam, params, w, wl=None):
    import torch
    sg = P.Scene.from_synth(scene)
    ws = P.Workspace()
    h, wd = cam.height, cam.width
    frame = dict(image=torch.empty((3, h, wd), device="cuda"), final_t=torch.empty((h, wd), device="cuda"),
                 l_iter=torch.empty((h, wd), dtype=torch.int32, device="cuda"))
    P.render(sg, cam, params, ws, **frame)
    dload = None if wl is None else torch.as_tensor(wl, dtype=torch.float32, device="cuda")
    g = P.render_backward(sg, cam, params, ws, frame, torch.as_tensor(w, dtype=torch.float32, device="cuda"),
                          dl_dload=dload)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in g.items()}, frame["image"].cpu().numpy()


def compare(g, o, what):
    for k in KEYS:
        scale = float(np.abs(o[k]).max())
        err = float(np.abs(g[k] - o[k]).max())
        say(f"{what} {k}: max |oracle| {scale:.3e}, max |diff| {err:.3e}")
        assert np.all(np.isfinite(g[k])), k
        assert err <= REL_TOL * max(scale, 1e-6), (what, k, err, scale)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["3sigma", "adaptive", "aabb"])
def test_gradients_match_the_oracle(P, mode):
    scene = f32(scene_small_sh3(300, seed=11))
    cam = camera_small(64, 48)
    prm = O.Params(cull=mode, background=(0.1, 0.2, 0.3))
    w = np.random.default_rng(5).normal(size=(3, cam.height, cam.width))
    say(f"300 G, SH3, 64x48, mode {mode}")
    g, img = gpu_grads(P, scene, cam, P.RenderParams(cull=mode, background=(0.1, 0.2, 0.3)), w)
    fwd = O.render_frame(scene, cam, prm)
    assert np.abs(img - fwd["image"]).max() <= 2e-4
    o = G.render_grad(scene, cam, prm, w, fwd)
    compare(g, o, f"mode {mode}")


def test_gradients_are_the_same_for_every_cull_mode(P):
    scene = f32(scene_small_sh3(300, seed=12))
    cam = camera_small(64, 64)
    w = np.random.default_rng(6).normal(size=(3, 64, 64))
    gs = [gpu_grads(P, scene, cam, P.RenderParams(cull=m), w)[0] for m in (0, 1, 2)]
    for k in KEYS:
        scale = float(np.abs(gs[0][k]).max())
        for other in gs[1:]:
            assert float(np.abs(other[k] - gs[0][k]).max()) <= 1e-5 * max(scale, 1e-6), k


def test_gradients_with_the_blend_cap_and_a_larger_scene(P):
    """The load-balancing cap (stop after K blends) and an orbit camera over a
    2000-Gaussian SH0 scene at 96x80."""
    scene = f32(scene_small(2000, seed=3))
    cam = camera_orbit(4.0, 20.0, 30.0, 96, 80, 60.0)
    prm = O.Params(cull=2, lb_cap=6)
    w = np.random.default_rng(8).normal(size=(3, 80, 96))
    g, _ = gpu_grads(P, scene, cam, P.RenderParams(cull=2, lb_cap=6), w)
    o = G.render_grad(scene, cam, prm, w)
    compare(g, o, "cap 6")


def test_autograd_function_gives_the_same_gradients(P):
    import torch
    scene = f32(scene_small_sh3(200, seed=13))
    cam = camera_small(48, 48)
    prm = P.RenderParams(cull=2)
    t = {k: torch.tensor(np.asarray(getattr(scene, k), dtype=np.float32), device="cuda", requires_grad=True)
         for k in KEYS}
    img = P.render_differentiable(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], cam, prm)
    w = torch.as_tensor(np.random.default_rng(9).normal(size=(3, 48, 48)), dtype=torch.float32, device="cuda")
    (img * w).sum().backward()
    ref, _ = gpu_grads(P, scene, cam, prm, w.cpu().numpy())
    for k in KEYS:
        got = t[k].grad.double().cpu().numpy()
        scale = float(np.abs(ref[k]).max())
        assert float(np.abs(got - ref[k]).max()) <= 1e-5 * max(scale, 1e-6), k


def test_backward_needs_the_matching_forward(P):
    import torch
    scene = P.Scene.from_synth(scene_small(100, seed=1))
    ws = P.Workspace()
    cam = camera_small(32, 32)
    frame = dict(image=torch.empty((3, 32, 32), device="cuda"), final_t=torch.empty((32, 32), device="cuda"),
                 l_iter=torch.empty((32, 32), dtype=torch.int32, device="cuda"))
    P.render(scene, cam, P.RenderParams(), ws, **frame)
    dl = torch.ones((3, 32, 32), device="cuda")
    with pytest.raises(P.AdrError):
        P.render_backward(scene, camera_small(32, 33), P.RenderParams(), ws, frame, dl)
    with pytest.raises(P.AdrError):
        P.render_backward(scene, cam, P.RenderParams(cull=0), ws, frame, dl)
    P.render_backward(scene, cam, P.RenderParams(), ws, frame, dl)
    torch.cuda.synchronize()


def test_gaussians_behind_the_camera_get_zero_gradients(P):
    """Every Gaussian behind the near plane: the frame is the background and
    every gradient element is written as zero."""
    import torch
    s = f32(scene_small_sh3(100, seed=14))
    s.means[:, 2] = -6.0  # camera at z = -4 looking along +z
    cam = camera_small(32, 32)
    prm = P.RenderParams(cull=2, background=(0.3, 0.2, 0.1))
    g, img = gpu_grads(P, s, cam, prm, np.ones((3, 32, 32)))
    for k in KEYS:
        assert not np.any(g[k]), k
    assert np.allclose(img, np.array([0.3, 0.2, 0.1])[:, None, None])


@pytest.mark.parametrize("mode", [0, 2], ids=["3sigma", "aabb"])
def test_load_term_gradients_match_the_oracle(P, mode):
    """adr_render_backward_load: dL/d(per-pixel load) through the blended alphas
    (slope 1), together with dL/dimage."""
    scene = f32(scene_small_sh3(300, seed=15))
    cam = camera_small(64, 48)
    rng = np.random.default_rng(10)
    w = rng.normal(size=(3, 48, 64))
    wl = rng.normal(size=(48, 64))
    say(f"load term, mode {mode}")
    g, _ = gpu_grads(P, scene, cam, P.RenderParams(cull=mode), w, wl)
    o = G.render_grad(scene, cam, O.Params(cull=mode), w, dl_dload=wl)
    compare(g, o, f"load mode {mode}")


@pytest.mark.parametrize("n_weak", [0, 1])
@pytest.mark.parametrize("mode", [0, 2], ids=["3sigma", "aabb"])
def test_gradients_on_the_stopped_pixel_scene(P, mode, n_weak):
    """The hand-placed scene of tests/stop_scene.py: pixels of the image's
    first quadrant stop at a wall with a Gaussian decided in FP64 only right
    behind it, the rest of their wave goes on. The backward walk must take
    the forward's decisions (stop, FP64-only blends) there too."""
    from tests.stop_scene import stop_scene
    scene, cam, _ = stop_scene(n_weak)
    scene = f32(scene)
    prm = O.Params(cull=mode)
    w = np.random.default_rng(9).normal(size=(3, cam.height, cam.width))
    say(f"stopped-pixel scene, {n_weak} weak walls, mode {mode}")
    g, img = gpu_grads(P, scene, cam, P.RenderParams(cull=mode), w)
    fwd = O.render_frame(scene, cam, prm)
    assert np.abs(img - fwd["image"]).max() <= 2e-4
    o = G.render_grad(scene, cam, prm, w, fwd)
    compare(g, o, f"stop scene {n_weak} mode {mode}")
