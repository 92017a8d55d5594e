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


def _tile_mask(cam, tiles):
    tx_n = (cam.width + 15) // 16
    keep = np.zeros((cam.height, cam.width), dtype=bool)
    for t in tiles:
        keep[(t // tx_n) * 16:(t // tx_n + 1) * 16, (t % tx_n) * 16:(t % tx_n + 1) * 16] = True
    return keep


def _oracle_piece(scene, cam, prm, tiles):
    """The forward oracle's lists and, on the given tiles, its per-pixel
    counters (all that the gradient oracle needs for a loss on those tiles)."""
    pre = O.preprocess(scene, cam, prm)
    rects = O.tile_rects(pre, cam, prm)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    r = O.render_image(pre, values, ranges, cam, prm, tiles=tiles)
    return dict(pre=pre, values=values, ranges=ranges, l_iter=r["l_iter"], l_blend=r["l_blend"],
                image=r["image"], done=r["done"], alpha_margin=r["alpha_margin"], t_margin=r["t_margin"])


def _elementwise(g, o, what, eps_frac=1e-5, rel=REL_TOL):
    """|g - o| <= rel |o| + eps, eps = eps_frac of the array's largest |o|:
    the FP32 sums behind each GPU element carry an absolute rounding error
    that the floor covers where the FP64 value is a nearly cancelling sum."""
    worst = {}
    for k in KEYS:
        scale = float(np.abs(o[k]).max())
        eps = eps_frac * max(scale, 1e-12)
        excess = np.abs(g[k] - o[k]) / (rel * np.abs(o[k]) + eps)
        worst[k] = float(excess.max())
        say(f"{what} {k}: max |oracle| {scale:.3e}, eps {eps:.2e}, worst |diff| / bound {worst[k]:.3f}")
        assert np.all(np.isfinite(g[k])), k
        assert worst[k] <= 1.0, (what, k, worst[k])
    return worst


@pytest.mark.slow
def test_c4_scale_gradients_per_element_and_central_differences(P):
    """The differentiation workload at its own scale: 500k Gaussians (SH
    degree 3) seen at 980x545 from the orbit, L1 loss against the render of a
    perturbed copy (means + N(0, 0.01), opacity logits + N(0, 0.2)). The loss
    is restricted to 24 seeded and the 8 heaviest tiles; every gradient
    element of every Gaussian matches the FP64 oracle within 1e-3 relative
    (plus a floor of 1e-5 of the array's largest value). Then 64 Gaussians of
    four seeded tiles: the GPU gradient of the loss on those tiles against
    central differences of the FP64 forward oracle (steps that change any
    blend decision are skipped)."""
    import torch
    from synth import scene_clusters, camera_orbit, Scene

    base = scene_clusters(500_000, seed=4)
    scene = f32(base)
    cam = camera_orbit(30.0, 20.0, 45.0, 980, 545, 60.0)
    rng = np.random.default_rng(40)
    target = Scene(base.means + rng.normal(0.0, 0.01, base.means.shape).astype(np.float32), base.log_scales,
                   base.quats, base.opacity_logits + rng.normal(0.0, 0.2, base.opacity_logits.shape).astype(np.float32),
                   base.sh, base.sh_degree)
    params = P.RenderParams(cull=2)
    prm = O.Params(cull=2)
    ws = P.Workspace()
    h, wd = cam.height, cam.width
    tgt = torch.empty((3, h, wd), device="cuda")
    st = P.Scene.from_synth(target)
    P.render(st, cam, params, ws, image=tgt)
    sg = P.Scene.from_synth(scene)
    frame = dict(image=torch.empty((3, h, wd), device="cuda"), final_t=torch.empty((h, wd), device="cuda"),
                 l_iter=torch.empty((h, wd), dtype=torch.int32, device="cuda"),
                 ranges=torch.empty((((wd + 15) // 16) * ((h + 15) // 16), 2), dtype=torch.int32, device="cuda"))
    P.render(sg, cam, params, ws, **frame)
    ranges = frame["ranges"].cpu().numpy().astype(np.int64)
    n_t = ranges.shape[0]
    tiles = np.unique(np.concatenate([np.argsort(ranges[:, 1] - ranges[:, 0])[-8:],
                                      np.random.default_rng(41).choice(n_t, 24, replace=False)]))
    say(f"C4: 500k G SH3 980x545, {tiles.size} tiles, longest list {int((ranges[:, 1] - ranges[:, 0]).max())}")
    w_l1 = torch.sign(frame["image"] - tgt).cpu().numpy().astype(np.float64)
    w = np.where(_tile_mask(cam, tiles)[None], w_l1, 0.0)
    g = P.render_backward(sg, cam, params, ws, frame, torch.as_tensor(w, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    g = {k: v.double().cpu().numpy() for k, v in g.items()}
    piece = _oracle_piece(scene, cam, prm, tiles)
    mask = piece["done"]
    assert np.abs(frame["image"].cpu().numpy()[:, mask] - piece["image"][:, mask]).max() <= 2e-4
    o = G.render_grad(scene, cam, prm, w, piece, tiles=tiles)
    _elementwise(g, o, "C4 tile subset")

    # central differences of the FP64 oracle on 64 Gaussians of four tiles,
    # evaluated on the scene restricted to the Gaussians of those tiles' lists
    # (their lists, in (depth, id) order, are the same there)
    fd_tiles = np.random.default_rng(42).choice(tiles, 4, replace=False)
    w_fd = np.where(_tile_mask(cam, fd_tiles)[None], w_l1, 0.0)
    g_fd = P.render_backward(sg, cam, params, ws, frame, torch.as_tensor(w_fd, dtype=torch.float32, device="cuda"))
    g_fd = {k: v.double().cpu().numpy() for k, v in g_fd.items()}
    vals = np.asarray(piece["values"], dtype=np.int64)
    ids = np.unique(np.concatenate([vals[ranges[t, 0]:ranges[t, 1]] for t in fd_tiles]))
    sub = Scene(*(np.array(getattr(scene, k)[ids], copy=True) for k in KEYS), scene.sh_degree)
    fd_mask = _tile_mask(cam, fd_tiles)

    def loss_and_decisions(sc):
        pc = _oracle_piece(sc, cam, prm, fd_tiles)
        return float(np.sum(w_fd[:, fd_mask] * pc["image"][:, fd_mask])), pc["l_iter"][fd_mask], pc["l_blend"][fd_mask]

    _, li0, lb0 = loss_and_decisions(sub)
    hit = np.nonzero(np.abs(g_fd["opacity_logits"][ids]) > 0)[0]
    picks = np.random.default_rng(43).choice(hit, min(64, hit.size), replace=False)
    slots = [("means", (0,)), ("log_scales", (1,)), ("quats", (2,)), ("opacity_logits", ()), ("sh", (1, 0)),
             ("means", (2,)), ("sh", (0, 1)), ("log_scales", (0,))]
    checked = skipped = 0
    eps = {k: 1e-5 * float(np.abs(g_fd[k]).max()) for k in KEYS}
    for n_pick, li in enumerate(picks):
        key, sub_idx = slots[n_pick % len(slots)]
        idx = (int(li),) + sub_idx
        arr = getattr(sub, key)
        step = 1e-5 * max(1.0, abs(float(arr[idx])))
        ls = []
        flipped = False
        for sgn in (1.0, -1.0):
            pert = Scene(*(np.array(getattr(sub, k), copy=True) for k in KEYS), sub.sh_degree)
            getattr(pert, key)[idx] += sgn * step
            val, li1, lb1 = loss_and_decisions(pert)
            flipped |= not (np.array_equal(li1, li0) and np.array_equal(lb1, lb0))
            ls.append(val)
        if flipped:
            skipped += 1
            continue
        fd = (ls[0] - ls[1]) / (2 * step)
        an = float(g_fd[key][(int(ids[li]),) + sub_idx])
        assert abs(fd - an) <= REL_TOL * abs(fd) + eps[key], (key, idx, fd, an)
        checked += 1
    say(f"central differences: {checked} checked, {skipped} skipped (a step changed a decision)")
    assert checked >= 48
    ws.close()
