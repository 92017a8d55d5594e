"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer outputs (tiles_touched, pair count, sorted keys and ids, tile ranges,
per-pixel load counters and their sums) must match bit for bit; images must
agree within 2e-4 per channel. Runs on an MI355X only."""
import math

import numpy as np
import pytest

import oracle as O
from synth import (Camera, scene_small, scene_needles, scene_clusters, scene_heavy, camera_small, camera_orbit,
                   camera_1080p, cameras_sweep)

pytestmark = pytest.mark.gpu

IMG_TOL = 2e-4
MARGIN = 1e-9  # oracle decisions closer than this to a threshold are ambiguous even in FP64


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08669_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def ws(P):
    return P.Workspace()


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_frame(P, ws, scene_gpu, cam, mode, debug=True, **kw):
    params = P.RenderParams(cull=mode, **kw)
    out = P.render_frame(scene_gpu, cam, params, ws=ws, debug=debug)
    res = {k: (to_np(v) if hasattr(v, "cpu") else v) for k, v in out.items() if k != "workspace"}
    for k in ("l_iter", "l_blend", "tiles_touched", "values", "ranges"):
        if k in res:
            res[k] = res[k].view(np.uint32)
    if "keys" in res:
        res["keys"] = res["keys"].view(np.uint64)
    return res


def gpu_frame_once(P, ws, scene_gpu, cam, mode, n_pairs_expected, **kw):
    """One adr_render call that writes every output, the sorted pairs into
    buffers sized from the oracle's pair count: when ws has not yet held a
    frame this large, this is the frame during which its buffers grow."""
    import torch
    w, h = int(cam.width), int(cam.height)
    tiles = ((w + 15) // 16) * ((h + 15) // 16)
    cap = max(int(n_pairs_expected), 1)
    out = dict(image=torch.empty((3, h, w), device="cuda"), final_t=torch.empty((h, w), device="cuda"),
               l_iter=torch.empty((h, w), dtype=torch.int32, device="cuda"),
               l_blend=torch.empty((h, w), dtype=torch.int32, device="cuda"),
               load_sums=torch.zeros(4, dtype=torch.int64, device="cuda"),
               load_stats=torch.zeros(4, dtype=torch.float64, device="cuda"),
               tiles_touched=torch.empty(max(scene_gpu.n, 1), dtype=torch.int32, device="cuda"),
               keys=torch.empty(cap, dtype=torch.int64, device="cuda"),
               values=torch.empty(cap, dtype=torch.int32, device="cuda"),
               ranges=torch.empty((tiles, 2), dtype=torch.int32, device="cuda"))
    n = P.render(scene_gpu, cam, P.RenderParams(cull=mode, **kw), ws, **out, pair_capacity=cap)
    res = {k: to_np(v) for k, v in out.items()}
    for k in ("l_iter", "l_blend", "tiles_touched", "values", "ranges"):
        res[k] = res[k].view(np.uint32)
    res["keys"] = res["keys"].view(np.uint64)[:n]
    res["values"] = res["values"][:n]
    res["tiles_touched"] = res["tiles_touched"][:scene_gpu.n]
    res["n_pairs"] = n
    return res


def check_no_bad_sort_indices(ws):
    assert ws.counters()["bad_sort_indices"] == 0


def oracle_params(mode, **kw):
    return O.Params(cull=mode, **kw)


def check_integer_stage(g, o, n):
    np.testing.assert_array_equal(g["tiles_touched"][:n], o["tiles_touched"], err_msg="tiles_touched")
    assert g["n_pairs"] == o["n_pairs"], (g["n_pairs"], o["n_pairs"])
    np.testing.assert_array_equal(g["keys"], o["keys"], err_msg="sorted keys")
    np.testing.assert_array_equal(g["values"], o["values"], err_msg="sorted ids")
    np.testing.assert_array_equal(g["ranges"].reshape(-1, 2), o["ranges"], err_msg="tile ranges")


def check_pixels(g, o, mask=None):
    """Image within IMG_TOL; counters exact except where the oracle's own
    decision margin is below MARGIN."""
    if mask is None:
        mask = np.ones(o["l_iter"].shape, dtype=bool)
    diff = np.abs(g["image"] - o["image"])[:, mask]
    assert diff.size == 0 or diff.max() <= IMG_TOL, f"image max |diff| {diff.max():.3e}"
    ambiguous = (o["alpha_margin"] < MARGIN) | (o["t_margin"] < MARGIN)
    ok = mask & ~ambiguous
    bad_b = int((g["l_blend"][ok] != o["l_blend"][ok]).sum())
    bad_i = int((g["l_iter"][ok] != o["l_iter"][ok]).sum())
    assert bad_b == 0 and bad_i == 0, f"load counters differ at {bad_b} / {bad_i} pixels"
    np.testing.assert_allclose(g["final_t"][mask], o["final_t"][mask], rtol=1e-3, atol=2e-6)
    return int(ambiguous.sum())


def check_load_sums(g, o):
    lb = o["l_blend"].astype(np.int64)
    li = o["l_iter"].astype(np.int64)
    expect = [lb.sum(), (lb * lb).sum(), li.sum(), (li * li).sum()]
    assert [int(v) for v in g["load_sums"]] == [int(v) for v in expect]
    if "load_stats" in g:  # Eq. 13, computed in the library from the exact sums
        want = list(O.load_stats(o["l_blend"])) + list(O.load_stats(o["l_iter"]))
        np.testing.assert_allclose(g["load_stats"], want, rtol=1e-12, atol=0)


@pytest.fixture(scope="module")
def small(P):
    s = scene_small(2000, seed=0)
    return s, P.Scene.from_synth(s), camera_small()


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["3sigma", "adaptive", "aabb"])
def test_small_scene_parity(P, ws, small, mode):
    s, sg, cam = small
    say(f"small scene 2000 G, 128x128, mode {mode}")
    g = gpu_frame(P, ws, sg, cam, mode)
    o = O.render_frame(s, cam, oracle_params(mode))
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)
    check_load_sums(g, o)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["3sigma", "adaptive", "aabb"])
def test_first_frame_on_a_fresh_workspace_matches_the_oracle(P, small, mode):
    """The frame during which a new workspace's buffers are allocated, read
    back from that same call (no second render): integer stage bit-exact,
    image and counters against the oracle, no out-of-range sort index."""
    s, sg, cam = small
    say(f"fresh workspace, small scene, mode {mode}")
    o = O.render_frame(s, cam, oracle_params(mode))
    fresh = P.Workspace()
    g = gpu_frame_once(P, fresh, sg, cam, mode, o["n_pairs"])
    check_no_bad_sort_indices(fresh)
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)
    check_load_sums(g, o)
    fresh.close()


def test_borrowed_scene_and_caller_allocator_give_the_same_frame(P, ws, small):
    """A scene that reads the caller's row-major device tensors in place
    (borrow) and a workspace whose arenas come from torch's caching allocator
    render bitwise the frame of a copied scene on a library workspace."""
    import torch
    s, sg, cam = small
    say("borrowed scene + torch allocator")
    ref = gpu_frame(P, ws, sg, cam, 2)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(s, k))).cuda()
         for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    sb = P.Scene(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], s.sh_degree, borrow=True)
    assert sb.bytes == 0
    wt = P.Workspace(allocator="torch")
    g = gpu_frame(P, wt, sb, cam, 2)
    for k in ("image", "final_t", "l_iter", "l_blend", "load_sums", "load_stats", "keys", "values", "ranges",
              "tiles_touched"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    wt.close()
    sb.close()


def test_reserved_workspace_allocates_nothing_while_rendering(P, small):
    """After adr_workspace_reserve for the frame's sizes, rendering the frame
    in every cull mode leaves the workspace's device bytes unchanged."""
    s, sg, cam = small
    o = O.render_frame(s, cam, oracle_params(0))
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    r = P.Workspace()
    r.reserve(s.n, o["n_pairs"], tiles)
    before = r.capacity_bytes
    # three frame slots, each sized for the frame
    assert before == 3 * P.Workspace.bytes_for(s.n, o["n_pairs"], tiles)
    for mode in (0, 1, 2):
        gpu_frame(P, r, sg, cam, mode, debug=False)
    assert r.capacity_bytes == before
    r.close()


@pytest.mark.parametrize("k", [2, 4, 8])
def test_alpha_low_sweep_parity(P, ws, small, k):
    """Larger alpha_low (the lossy speed-up of Sec. 5.1.2): the adaptive and
    AABB extents shrink with it and the blend skips more entries, and every
    output still matches the oracle run at the same alpha_low; 3-sigma and
    AABB give the same image."""
    s, sg, cam = small
    a = k / 255.0
    say(f"small scene 2000 G, 128x128, alpha_low {k}/255")
    o = O.render_frame(s, cam, oracle_params(2, alpha_low=a))
    g = gpu_frame(P, ws, sg, cam, 2, alpha_low=a)
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)
    check_load_sums(g, o)
    g3 = gpu_frame(P, ws, sg, cam, 0, debug=False, alpha_low=a)
    assert np.array_equal(g3["image"], g["image"])
    assert np.array_equal(g3["l_blend"], g["l_blend"])


@pytest.mark.parametrize("mode", [0, 2], ids=["3sigma", "aabb"])
def test_needle_scene_parity(P, ws, mode):
    """Long thin Gaussians at every angle (projected axis ratios up to ~2600):
    the FP32 exponent's error bounds must keep every decision exact."""
    s = scene_needles(1500, seed=2)
    cam = camera_small(128, 128)
    say(f"needle scene 1500 G, 128x128, mode {mode}")
    g = gpu_frame(P, ws, P.Scene.from_synth(s), cam, mode)
    o = O.render_frame(s, cam, oracle_params(mode))
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)
    check_load_sums(g, o)


@pytest.mark.parametrize("n_weak", [0, 1])
@pytest.mark.parametrize("mode", [0, 2], ids=["3sigma", "aabb"])
def test_stopped_pixels_blend_nothing_more(P, ws, mode, n_weak):
    """Pixels that stop at a wall while their quadrant goes on, with a
    Gaussian decided in FP64 only right after the stop and a Gaussian 0 that
    reaches them (tests/stop_scene.py): their colour, transmittance and
    counters end at the stop, with the stop on either of the blend loop's two
    alternating steps (n_weak 0 and 1)."""
    from tests.stop_scene import stop_scene
    s, cam, _ = stop_scene(n_weak)
    say(f"stopped-pixel scene, {n_weak} weak walls, mode {mode}")
    g = gpu_frame(P, ws, P.Scene.from_synth(s), cam, mode)
    o = O.render_frame(s, cam, oracle_params(mode))
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)
    check_load_sums(g, o)


def test_small_scene_modes_render_bitwise_identical(P, ws, small):
    _, sg, cam = small
    say("mode invariance, small scene")
    outs = [gpu_frame(P, ws, sg, cam, m, debug=False) for m in (0, 1, 2)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o["image"], outs[0]["image"])
        np.testing.assert_array_equal(o["l_blend"], outs[0]["l_blend"])
        np.testing.assert_array_equal(o["final_t"], outs[0]["final_t"])
    assert np.all(outs[0]["l_iter"] >= outs[1]["l_iter"]) and np.all(outs[1]["l_iter"] >= outs[2]["l_iter"])
    assert outs[0]["n_pairs"] > outs[1]["n_pairs"] > outs[2]["n_pairs"]


def test_ablation_flags_keep_the_output(P, ws, small):
    """Disabling the render-side quadrant cull changes no output bit;
    disabling the FP64 bands keeps the image within tolerance."""
    s, sg, cam = small
    say("ablation flags")
    ref = gpu_frame(P, ws, sg, cam, 2, debug=False)
    nq = gpu_frame(P, ws, sg, cam, 2, debug=False, flags=P.ADR_FLAG_NO_QUAD_CULL)
    for k in ("image", "final_t", "l_iter", "l_blend", "load_sums"):
        np.testing.assert_array_equal(nq[k], ref[k], err_msg=k)
    nb = gpu_frame(P, ws, sg, cam, 2, debug=False, flags=P.ADR_FLAG_NO_EXACT_BAND)
    assert np.abs(nb["image"] - ref["image"]).max() <= IMG_TOL


def test_ragged_image_and_count(P, ws):
    s = scene_small(2001, seed=5)
    cam = camera_small(130, 70)  # 9 x 5 tiles, partial last column and row
    say("ragged 2001 G, 130x70")
    sg = P.Scene.from_synth(s)
    for mode in (0, 2):
        g = gpu_frame(P, ws, sg, cam, mode, background=(0.1, 0.2, 0.3))
        o = O.render_frame(s, cam, oracle_params(mode, background=(0.1, 0.2, 0.3)))
        check_integer_stage(g, o, s.n)
        check_pixels(g, o)
        check_load_sums(g, o)


def test_sh_degree3_scene_parity(P, ws):
    s = scene_clusters(40_000, seed=3)
    cam = camera_orbit(30.0, 20.0, 45.0, 320, 240)
    say("SH3 40k G, 320x240")
    sg = P.Scene.from_synth(s)
    g = gpu_frame(P, ws, sg, cam, 2)
    o = O.render_frame(s, cam, oracle_params(2))
    check_integer_stage(g, o, s.n)
    check_pixels(g, o)


def test_pipelined_frames_match_single_frames(P):
    """Consecutive adr_render calls on one workspace take its three frame
    slots in turn, and a frame's stages up to the tile order run on its
    slot's side stream, overlapping the early stages and the blend of the
    frames before it. Ten frames of three different scenes and image sizes,
    ordered so that every slot renders all three (its arenas grow between
    frames), are enqueued back to back, each into its own outputs, with no
    synchronisation; each must equal, bit for bit, the same frame rendered
    alone on a fresh workspace. The last two also run with the timing flag."""
    import torch
    cfgs = [(scene_clusters(40_000, seed=3), camera_orbit(30.0, 20.0, 45.0, 320, 240), 2),
            (scene_small(2000, seed=0), camera_small(), 0),
            (scene_clusters(200_000, seed=6), camera_orbit(30.0, 25.0, 120.0, 640, 480), 1)]
    gpu_scenes = [P.Scene.from_synth(c[0]) for c in cfgs]

    def outputs(cam):
        h, w = cam.height, cam.width
        return dict(image=torch.empty((3, h, w), device="cuda"), final_t=torch.empty((h, w), device="cuda"),
                    l_iter=torch.empty((h, w), dtype=torch.int32, device="cuda"),
                    l_blend=torch.empty((h, w), dtype=torch.int32, device="cuda"),
                    load_sums=torch.zeros(4, dtype=torch.int64, device="cuda"))

    seq = [0, 1, 2, 1, 2, 0, 2, 0, 1, 0]  # frame i in slot i mod 3
    ws = P.Workspace()
    got = []
    for i, k in enumerate(seq):
        _, cam, mode = cfgs[k]
        out = outputs(cam)
        flags = P.ADR_FLAG_TIMING if i >= len(seq) - 2 else 0
        P.render(gpu_scenes[k], cam, P.RenderParams(cull=mode, flags=flags), ws, **out)
        got.append(out)
    torch.cuda.synchronize()
    for i, k in enumerate(seq):
        _, cam, mode = cfgs[k]
        ref = outputs(cam)
        fresh = P.Workspace()
        P.render(gpu_scenes[k], cam, P.RenderParams(cull=mode), fresh, **ref)
        torch.cuda.synchronize()
        for name in ref:
            assert torch.equal(got[i][name], ref[name]), (i, k, name)
        fresh.close()
    say(f"pipelined: {len(seq)} frames bitwise equal to single frames")
    ws.close()


def test_load_balancing_cap_parity(P, ws, small):
    s, sg, cam = small
    for k in (1, 3):
        say(f"load-balancing cap K={k}")
        g = gpu_frame(P, ws, sg, cam, 2, lb_cap=k)
        o = O.render_frame(s, cam, oracle_params(2, lb_cap=k))
        check_pixels(g, o)
        check_load_sums(g, o)
        assert g["l_blend"].max() <= k


def test_degenerate_scenes(P, ws):
    cam = camera_small(64, 48)
    say("empty scene")
    empty = scene_small(0, seed=0)
    g = gpu_frame(P, ws, P.Scene.from_synth(empty), cam, 2, background=(0.2, 0.4, 0.6))
    assert g["n_pairs"] == 0
    for c, v in enumerate((0.2, 0.4, 0.6)):
        assert np.all(g["image"][c] == np.float32(v))
    assert np.all(g["final_t"] == 1) and g["l_iter"].max() == 0
    say("single Gaussian")
    one = scene_small(1, seed=4)
    one.means[:] = 0
    one.log_scales[:] = -1.5
    one.opacity_logits[:] = 2.0
    g = gpu_frame(P, ws, P.Scene.from_synth(one), cam, 2)
    o = O.render_frame(one, cam, oracle_params(2))
    check_integer_stage(g, o, 1)
    check_pixels(g, o)
    say("all opacities below alpha_low")
    low = scene_small(300, seed=6)
    low.opacity_logits[:] = np.float32(math.log((0.9 / 255) / (1 - 0.9 / 255)))
    for mode in (0, 1, 2):
        g = gpu_frame(P, ws, P.Scene.from_synth(low), cam, mode)
        o = O.render_frame(low, cam, oracle_params(mode))
        check_integer_stage(g, o, low.n)
        assert np.all(g["image"] == 0) and g["l_blend"].max() == 0
    say("everything behind the camera")
    behind = scene_small(300, seed=7)
    behind.means[:, 2] = -10.0
    g = gpu_frame(P, ws, P.Scene.from_synth(behind), cam, 0)
    assert g["n_pairs"] == 0 and np.all(g["tiles_touched"] == 0)


def test_pair_capacity_too_small_reports_workspace_error(P, ws, small):
    import torch
    _, sg, cam = small
    say("pair capacity error path")
    img = torch.empty((3, cam.height, cam.width), device="cuda")
    keys = torch.empty(10, dtype=torch.int64, device="cuda")
    vals = torch.empty(10, dtype=torch.int32, device="cuda")
    with pytest.raises(P.AdrError) as ei:
        P.render(sg, cam, P.RenderParams(), ws, img, keys=keys, values=vals, pair_capacity=10)
    assert ei.value.status == -5 and ei.value.n_pairs > 10


def test_repeat_runs_are_bitwise_identical(P, ws, small):
    _, sg, cam = small
    say("determinism")
    a = gpu_frame(P, ws, sg, cam, 2)
    b = gpu_frame(P, ws, sg, cam, 2)
    for k in ("image", "final_t", "l_iter", "l_blend", "keys", "values", "ranges", "load_sums"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.slow
def test_headline_scale_integer_stage_and_sampled_tiles(P, ws):
    """1M Gaussians, SH3, 1920x1080: the full integer stage bit-exact, and the
    image and counters on 48 seeded tiles against the oracle."""
    s = scene_clusters(1_000_000, seed=0)
    cam = camera_1080p()
    sg = P.Scene.from_synth(s)
    pre = O.preprocess(s, cam, O.Params())
    rng = np.random.default_rng(11)
    tx_n, ty_n = O.n_tiles(cam)
    for mode in (0, 2):
        say(f"1M G 1080p mode {mode}")
        g = gpu_frame(P, ws, sg, cam, mode)
        params = oracle_params(mode)
        rects = O.tile_rects(pre, cam, params)
        keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
        ranges = O.tile_ranges(keys, cam)
        o = dict(tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size), keys=keys, values=values,
                 ranges=ranges)
        check_integer_stage(g, o, s.n)
        busy = np.argsort(ranges[:, 1] - ranges[:, 0])[-16:]
        tiles = np.unique(np.concatenate([rng.choice(tx_n * ty_n, 32, replace=False), busy]))
        r = O.render_image(pre, values, ranges, cam, params, tiles=tiles)
        n_amb = check_pixels(g, r, mask=r["done"])
        say(f"  pairs {g['n_pairs']}  sampled tiles {tiles.size}  ambiguous pixels {n_amb}")
    say("1M G 1080p: 3-sigma and AABB images bitwise identical")
    a = gpu_frame(P, ws, sg, cam, 0, debug=False)
    b = gpu_frame(P, ws, sg, cam, 2, debug=False)
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["l_blend"], b["l_blend"])


@pytest.mark.slow
def test_4k_frame_integer_stage_and_sampled_tiles(P, ws):
    """The largest frame size of the workloads: 1M Gaussians (SH3, seed 1),
    3840x2160 from a 14 m orbit so that the scene reaches every image corner
    (~9.8M pairs, 32400 tiles). AABB: the integer stage bit-exact, then the
    image and counters on the four corner tiles, the 16 busiest and 32 seeded
    tiles against the oracle; the 3-sigma image bitwise the AABB one."""
    s = scene_clusters(1_000_000, seed=1)
    cam = camera_orbit(14.0, 35.0, 200.0, 3840, 2160)
    sg = P.Scene.from_synth(s)
    pre = O.preprocess(s, cam, O.Params())
    params = oracle_params(2)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    say("1M G 3840x2160 AABB")
    g = gpu_frame(P, ws, sg, cam, 2)
    o = dict(tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size), keys=keys, values=values, ranges=ranges)
    check_integer_stage(g, o, s.n)
    tx_n, ty_n = O.n_tiles(cam)
    corners = np.array([0, tx_n - 1, (ty_n - 1) * tx_n, tx_n * ty_n - 1])
    assert (ranges[corners, 1] > ranges[corners, 0]).all()  # the scene reaches every corner
    busy = np.argsort(ranges[:, 1] - ranges[:, 0])[-16:]
    rng = np.random.default_rng(13)
    tiles = np.unique(np.concatenate([rng.choice(tx_n * ty_n, 32, replace=False), busy, corners]))
    r = O.render_image(pre, values, ranges, cam, params, tiles=tiles)
    n_amb = check_pixels(g, r, mask=r["done"])
    say(f"  pairs {g['n_pairs']}  sampled tiles {tiles.size}  ambiguous pixels {n_amb}")
    # The 3-sigma frame next, on the same workspace: twice the pairs, so its
    # pair and sort buffers grow during this very call. Its integer stage
    # bit-exact against the oracle, its image bitwise the AABB one.
    params3 = oracle_params(0)
    rects3 = O.tile_rects(pre, cam, params3)
    keys3, values3, _ = O.duplicate_and_sort(pre, rects3, cam)
    say(f"1M G 3840x2160 3-sigma on the same workspace, {keys3.size} pairs (buffers grow)")
    b = gpu_frame_once(P, ws, sg, cam, 0, keys3.size)
    check_no_bad_sort_indices(ws)
    o3 = dict(tiles_touched=rects3["tiles_touched"], n_pairs=int(keys3.size), keys=keys3, values=values3,
              ranges=O.tile_ranges(keys3, cam))
    check_integer_stage(b, o3, s.n)
    np.testing.assert_array_equal(b["image"], g["image"])
    np.testing.assert_array_equal(b["l_blend"], g["l_blend"])


@pytest.mark.slow
def test_4k_frame_3sigma_integer_stage(P, ws):
    """The same 4K frame with 3-sigma culling: ~20.4M Gaussian-tile pairs,
    the largest pair count of the tests. Tiles touched, pair count, sorted
    keys and ids and tile ranges bit-exact against the oracle, and the image
    bitwise the AABB one."""
    s = scene_clusters(1_000_000, seed=1)
    cam = camera_orbit(14.0, 35.0, 200.0, 3840, 2160)
    sg = P.Scene.from_synth(s)
    pre = O.preprocess(s, cam, O.Params())
    params = oracle_params(0)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    say(f"1M G 3840x2160 3-sigma on a fresh workspace, {keys.size} pairs (buffers grow)")
    fresh = P.Workspace()
    g = gpu_frame_once(P, fresh, sg, cam, 0, keys.size)
    check_no_bad_sort_indices(fresh)
    o = dict(tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size), keys=keys, values=values, ranges=ranges)
    check_integer_stage(g, o, s.n)
    a = gpu_frame(P, fresh, sg, cam, 2, debug=False)
    np.testing.assert_array_equal(g["image"], a["image"])
    fresh.close()


def test_frame_of_more_than_65536_tiles(P, ws):
    """4608x4096 (73728 tiles, 50k Gaussians), a tile grid larger than any
    of the workloads': the integer stage bit-exact, 34 sampled tiles
    (corners, busiest, seeded) against the oracle, and the frame's l_iter sum
    equal to the one in its load sums."""
    s = scene_clusters(50_000, seed=4)
    cam = camera_orbit(14.0, 35.0, 120.0, 4608, 4096)
    sg = P.Scene.from_synth(s)
    pre = O.preprocess(s, cam, O.Params())
    params = oracle_params(2)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    tx_n, ty_n = O.n_tiles(cam)
    assert tx_n * ty_n > 65536
    say("50k G 4608x4096 AABB")
    g = gpu_frame(P, ws, sg, cam, 2)
    o = dict(tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size), keys=keys, values=values, ranges=ranges)
    check_integer_stage(g, o, s.n)
    busy = np.argsort(ranges[:, 1] - ranges[:, 0])[-8:]
    rng = np.random.default_rng(14)
    tiles = np.unique(np.concatenate([rng.choice(tx_n * ty_n, 24, replace=False), busy, [0, tx_n * ty_n - 1]]))
    r = O.render_image(pre, values, ranges, cam, params, tiles=tiles)
    check_pixels(g, r, mask=r["done"])
    assert int(g["load_sums"][2]) == int(g["l_iter"].astype(np.int64).sum())


@pytest.mark.slow
def test_load_imbalanced_scene_exact_and_capped(P, ws):
    """3M Gaussians with 20% in 8 dense clusters, 1600x1040, first pose of the
    32-pose sweep (tile lists up to ~76k entries): the AABB integer stage
    bit-exact, then the exact and the capped blend on 40 sampled tiles (the 8
    heaviest and 32 seeded). The cap is K = ceil(mean + 2 std) of l_blend over
    the covered pixels of the oracle's sampled tiles."""
    s = scene_heavy(3_000_000, seed=0)
    cam = cameras_sweep(32)[0]
    sg = P.Scene.from_synth(s)
    pre = O.preprocess(s, cam, O.Params())
    params = oracle_params(2)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    say("3M G 1600x1040 AABB exact")
    g = gpu_frame(P, ws, sg, cam, 2)
    o = dict(tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size), keys=keys, values=values, ranges=ranges)
    check_integer_stage(g, o, s.n)
    tx_n, ty_n = O.n_tiles(cam)
    rng = np.random.default_rng(12)
    busy = np.argsort(ranges[:, 1] - ranges[:, 0])[-8:]
    tiles = np.unique(np.concatenate([rng.choice(tx_n * ty_n, 32, replace=False), busy]))
    r = O.render_image(pre, values, ranges, cam, params, tiles=tiles)
    check_pixels(g, r, mask=r["done"])
    covered = r["done"] & (r["l_blend"] > 0)
    lb = r["l_blend"][covered].astype(np.float64)
    k = int(math.ceil(lb.mean() + 2.0 * lb.std()))
    say(f"  pairs {g['n_pairs']}  cap K = {k}")
    gc = gpu_frame(P, ws, sg, cam, 2, lb_cap=k)
    rc = O.render_image(pre, values, ranges, cam, oracle_params(2, lb_cap=k), tiles=tiles)
    check_pixels(gc, rc, mask=rc["done"])
    assert gc["l_blend"].max() <= k
