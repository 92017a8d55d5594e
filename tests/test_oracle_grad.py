"""Pins of the gradient oracle (oracle/adr_grad.py) against things other than
itself: central finite differences of the forward oracle's image, the
lossless property of the cull modes (Sec. 4: the adaptive radius and the AABB
leave every pixel's blend list unchanged, so the gradient is the same), and
the trivial cases (nothing reaches a pixel; Gaussians behind the camera)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import adr_grad as G
from synth import Scene, scene_small_sh3, camera_small

KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def sh3_scene(n, seed):
    return scene_small_sh3(n, seed=seed)


def perturbed(scene, key, idx, h):
    arrs = {k: np.array(getattr(scene, k), dtype=np.float64, copy=True) for k in KEYS}
    arrs[key][idx] += h
    return Scene(arrs["means"], arrs["log_scales"], arrs["quats"], arrs["opacity_logits"], arrs["sh"],
                 scene.sh_degree)


def test_gradient_matches_central_differences():
    scene = sh3_scene(40, seed=5)
    cam = camera_small(40, 32)
    prm = O.Params(cull=O.CULL_AABB, background=(0.2, 0.3, 0.1))
    rng = np.random.default_rng(1)
    w = rng.normal(size=(3, cam.height, cam.width))
    fwd = O.render_frame(scene, cam, prm)
    # no decision within reach of the perturbations below
    assert fwd["alpha_margin"].min() > 1e-5 and fwd["t_margin"].min() > 1e-5
    assert fwd["l_blend"].max() >= 3  # pixels that blend several Gaussians
    g = G.render_grad(scene, cam, prm, w, fwd)
    assert abs(g["loss"] - G.loss_of(scene, cam, prm, w)) < 1e-12 * max(1.0, abs(g["loss"]))
    # Gaussians that reach some pixel
    hit = np.unique(np.asarray(fwd["values"], dtype=np.int64))
    checked = 0
    for key in KEYS:
        arr = np.asarray(getattr(scene, key))
        for _ in range(10):
            gi = int(rng.choice(hit))
            idx = (gi,) + tuple(int(rng.integers(0, d)) for d in arr.shape[1:])
            h = 1e-7 * max(1.0, abs(float(arr[idx])))
            fd = (G.loss_of(perturbed(scene, key, idx, h), cam, prm, w)
                  - G.loss_of(perturbed(scene, key, idx, -h), cam, prm, w)) / (2 * h)
            an = float(g[key][idx])
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (key, idx, fd, an)
            checked += 1
    assert checked == 50


def test_gradient_is_the_same_for_every_cull_mode():
    scene = sh3_scene(60, seed=2)
    cam = camera_small(48, 40)
    w = np.random.default_rng(3).normal(size=(3, cam.height, cam.width))
    grads = [G.render_grad(scene, cam, O.Params(cull=m), w) for m in (O.CULL_3SIGMA, O.CULL_ADAPTIVE, O.CULL_AABB)]
    for k in KEYS:
        scale = max(1.0, float(np.abs(grads[0][k]).max()))
        for other in grads[1:]:
            assert np.abs(other[k] - grads[0][k]).max() <= 1e-12 * scale, k
    assert len({round(gr["loss"], 12) for gr in grads}) == 1


def test_gradient_of_an_empty_frame_is_zero():
    """Every opacity far below alpha_low: no pixel blends anything, the image is
    the background and L = sum(w * bg)."""
    scene = sh3_scene(30, seed=4)
    scene.opacity_logits[:] = -12.0
    cam = camera_small(32, 32)
    prm = O.Params(cull=O.CULL_3SIGMA, background=(0.5, 0.25, 1.0))
    w = np.random.default_rng(0).normal(size=(3, 32, 32))
    g = G.render_grad(scene, cam, prm, w)
    for k in KEYS:
        assert not np.any(g[k]), k
    assert math.isclose(g["loss"], float((w * np.array(prm.background)[:, None, None]).sum()), rel_tol=1e-12)


def test_gaussians_behind_the_camera_get_no_gradient():
    scene = sh3_scene(30, seed=6)
    behind = np.arange(0, 30, 3)
    scene.means[behind, 2] = -6.0  # camera at z = -4 looking along +z
    cam = camera_small(40, 40)
    w = np.random.default_rng(2).normal(size=(3, 40, 40))
    g = G.render_grad(scene, cam, O.Params(), w)
    for k in KEYS:
        assert not np.any(g[k][behind]), k
    assert np.any(g["means"])


def test_load_surrogate_gradient_matches_central_differences():
    """The load term: L = sum(w * image) + sum(wl * A) with A the per-pixel
    sum of the blended alphas (computed here by a NumPy loop over pixels)."""
    scene = sh3_scene(30, seed=8)
    cam = camera_small(32, 24)
    prm = O.Params(cull=O.CULL_AABB)
    rng = np.random.default_rng(4)
    w = rng.normal(size=(3, cam.height, cam.width))
    wl = rng.normal(size=(cam.height, cam.width))
    fwd = O.render_frame(scene, cam, prm)
    assert fwd["alpha_margin"].min() > 1e-5 and fwd["t_margin"].min() > 1e-5
    g = G.render_grad(scene, cam, prm, w, fwd, dl_dload=wl)

    def total(sc):
        return G.loss_of(sc, cam, prm, w) + float(np.sum(wl * G.blended_alpha_sum(sc, cam, prm)))

    assert abs(g["loss"] - total(scene)) < 1e-11 * max(1.0, abs(g["loss"]))
    hit = np.unique(np.asarray(fwd["values"], dtype=np.int64))
    for key in ("means", "log_scales", "quats", "opacity_logits"):
        arr = np.asarray(getattr(scene, key))
        for _ in range(4):
            gi = int(rng.choice(hit))
            idx = (gi,) + tuple(int(rng.integers(0, d)) for d in arr.shape[1:])
            h = 1e-7 * max(1.0, abs(float(arr[idx])))
            fd = (total(perturbed(scene, key, idx, h)) - total(perturbed(scene, key, idx, -h))) / (2 * h)
            an = float(g[key][idx])
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (key, idx, fd, an)


def test_tile_subset_gives_the_full_gradient_when_other_weights_vanish():
    """render_grad restricted to some tiles equals the full-frame gradient
    when the loss weights are zero on every other tile (those tiles' terms
    are exactly zero), and it refuses weights outside the given tiles."""
    scene = sh3_scene(120, seed=8)
    cam = camera_small(64, 48)
    prm = O.Params(cull=O.CULL_AABB)
    fwd = O.render_frame(scene, cam, prm)
    tx_n, ty_n = O.n_tiles(cam)
    tiles = [1, 5, 6, 10]
    w = np.zeros((3, cam.height, cam.width))
    rng = np.random.default_rng(3)
    for t in tiles:
        ys = slice((t // tx_n) * 16, (t // tx_n + 1) * 16)
        xs = slice((t % tx_n) * 16, (t % tx_n + 1) * 16)
        w[:, ys, xs] = rng.normal(size=w[:, ys, xs].shape)
    full = G.render_grad(scene, cam, prm, w, fwd)
    part = G.render_grad(scene, cam, prm, w, fwd, tiles=tiles)
    for k in KEYS:
        np.testing.assert_allclose(part[k], full[k], rtol=1e-12, atol=1e-15)
    assert any(np.abs(full[k]).max() > 0 for k in KEYS)
    with pytest.raises(AssertionError):
        G.render_grad(scene, cam, prm, w, fwd, tiles=tiles[:2])
