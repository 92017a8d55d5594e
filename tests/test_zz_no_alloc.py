"""adr_render_noalloc, the entry point that allocates nothing (its workspace
is carved from the library's fixed device scratch), against adr_render on
the same inputs: the same kernels in the same launch configuration, so every
output must be bitwise the same. Two calls in a row, the second on a smaller
scene and image, then the size limits. Runs on an MI355X only."""
import numpy as np
import pytest

from synth import Scene, camera_orbit, camera_pinhole, camera_small, scene_clusters, scene_small

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08669_amd as P
    P.load()
    return P


def outputs(cam, n, pair_cap):
    import torch
    w, h = int(cam.width), int(cam.height)
    tiles = ((w + 15) // 16) * ((h + 15) // 16)
    return dict(
        image=torch.full((3, h, w), -1.0, device="cuda"),
        final_t=torch.full((h, w), -1.0, device="cuda"),
        l_iter=torch.full((h, w), -1, dtype=torch.int32, device="cuda"),
        l_blend=torch.full((h, w), -1, dtype=torch.int32, device="cuda"),
        load_sums=torch.zeros(4, dtype=torch.int64, device="cuda"),
        load_stats=torch.zeros(4, dtype=torch.float64, device="cuda"),
        tiles_touched=torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda"),
        ranges=torch.full((tiles, 2), -1, dtype=torch.int32, device="cuda"),
        keys=torch.full((pair_cap,), -1, dtype=torch.int64, device="cuda"),
        values=torch.full((pair_cap,), -1, dtype=torch.int32, device="cuda"),
    )


def compare(P, scene_host, cam, mode, label):
    """adr_render (own workspace) and adr_render_noalloc on the same scene and
    camera with every output requested; all must be bitwise equal."""
    import torch
    sg = P.Scene.from_synth(scene_host)
    params = P.RenderParams(cull=mode)
    ws = P.Workspace()
    probe = outputs(cam, scene_host.n, 1)
    n_pairs = P.render(sg, cam, params, ws, image=probe["image"])
    say(f"{label}: {scene_host.n} Gaussians, {cam.width}x{cam.height}, {n_pairs} pairs")
    ref = outputs(cam, scene_host.n, max(n_pairs, 1))
    assert P.render(sg, cam, params, ws, **ref, pair_capacity=max(n_pairs, 1)) == n_pairs
    got = outputs(cam, scene_host.n, max(n_pairs, 1))
    assert P.render_noalloc(sg, cam, params, **got, pair_capacity=max(n_pairs, 1)) == n_pairs
    torch.cuda.synchronize()
    for k in ref:
        a, b = ref[k], got[k]
        if k in ("keys", "values"):
            a, b = a[:n_pairs], b[:n_pairs]
        if k == "tiles_touched":
            a, b = a[:scene_host.n], b[:scene_host.n]
        if a.dtype.is_floating_point:
            d = float((a - b).abs().max()) if a.numel() else 0.0
            assert d <= 2e-4, (label, k, d)
        assert torch.equal(a, b), (label, k)
    assert float(got["image"].abs().sum()) > 0.0  # something was drawn
    ws.close()
    sg.close()
    return n_pairs


def test_noalloc_matches_adr_render_on_two_calls_in_a_row(P):
    """A 40k-Gaussian SH3 cluster scene at 640x360, then (smaller in both
    Gaussians and image) the 2000-Gaussian parity scene at 128x128: the
    second call reuses the scratch that still holds the first call's data."""
    big = scene_clusters(40_000, seed=3)
    cam_big = camera_orbit(30.0, 20.0, 35.0, 640, 360)
    p1 = compare(P, big, cam_big, P.ADR_CULL_AABB, "first call")
    small = scene_small(2000, seed=0)
    p2 = compare(P, small, camera_small(), P.ADR_CULL_3SIGMA, "second call")
    assert p2 < p1


def test_noalloc_rejects_frames_beyond_its_scratch(P):
    """Too many tiles: rejected before anything is enqueued. Too many pairs:
    ADR_E_WORKSPACE after Preprocess with the frame's pair count. A normal
    call afterwards still matches adr_render."""
    import torch
    small = scene_small(200, seed=1)
    sg = P.Scene.from_synth(small)
    huge = camera_small(65535, 65535)  # 16.8M tiles: their arrays alone exceed the scratch
    dummy = torch.zeros(1, device="cuda")
    with pytest.raises(P.AdrError) as ei:
        P.render_noalloc(sg, huge, P.RenderParams(), image=dummy)
    assert ei.value.status == -5 and "tiles" in str(ei.value)
    sg.close()

    # 300 Gaussians 4 m in front of the camera with 2 m standard deviation:
    # every one covers all 65536 tiles of a 4096 x 4096 frame (3-sigma)
    rng = np.random.default_rng(7)
    n = 300
    wide = Scene(means=(rng.standard_normal((n, 3)) * 0.01).astype(np.float32),
                 log_scales=np.full((n, 3), np.log(2.0), dtype=np.float32),
                 quats=np.tile(np.array([1.0, 0.0, 0.0, 0.0], dtype=np.float32), (n, 1)),
                 opacity_logits=np.full(n, 3.0, dtype=np.float32),
                 sh=np.zeros((n, 1, 3), dtype=np.float32), sh_degree=0)
    cam = camera_pinhole([0.0, 0.0, -4.0], [0.0, 0.0, 0.0], 4096, 4096, 60.0)
    sg = P.Scene.from_synth(wide)
    out = dict(image=torch.empty((3, 4096, 4096), device="cuda"))
    with pytest.raises(P.AdrError) as ei:
        P.render_noalloc(sg, cam, P.RenderParams(cull=P.ADR_CULL_3SIGMA), **out)
    assert ei.value.status == -5
    assert ei.value.n_pairs == n * 65536, ei.value.n_pairs
    scratch = P.noalloc_scratch_bytes()
    assert ei.value.n_pairs * 16 > scratch - 65536 * 141
    say(f"rejected {ei.value.n_pairs} pairs: {ei.value}")
    sg.close()
    del out
    compare(P, scene_small(2000, seed=2), camera_small(96, 80), P.ADR_CULL_ADAPTIVE, "after the rejections")
