"""Serving (adr_server: resident scenes, continuous batching). Every frame of
a mixed stream of requests must be bitwise the frame adr_render gives for the
same request alone, the server must actually blend several frames in one
launch, and admission must respect the memory budget. Runs on an MI355X
only."""
import numpy as np
import pytest

from synth import scene_small, scene_clusters, camera_small, camera_orbit

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-server] {msg}", flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08669_amd as P
    P.load()
    return P


def outputs(cam, device="cuda"):
    import torch
    h, w = cam.height, cam.width
    return dict(image=torch.empty((3, h, w), device=device), final_t=torch.empty((h, w), device=device),
                l_iter=torch.empty((h, w), dtype=torch.int32, device=device),
                l_blend=torch.empty((h, w), dtype=torch.int32, device=device),
                load_sums=torch.zeros(4, dtype=torch.int64, device=device),
                load_stats=torch.zeros(4, dtype=torch.float64, device=device))


def _requests(P):
    scenes = [P.Scene.from_synth(scene_small(2000, seed=0)), P.Scene.from_synth(scene_clusters(40_000, seed=3)),
              P.Scene.from_synth(scene_clusters(200_000, seed=5))]
    cams = [camera_small(128, 128), camera_small(130, 70), camera_orbit(30.0, 20.0, 45.0, 320, 240),
            camera_orbit(30.0, 25.0, 120.0, 640, 480), camera_orbit(20.0, 15.0, 300.0, 1280, 720)]
    reqs = []
    for i in range(24):
        sg = scenes[i % len(scenes)]
        cam = cams[(i * 7) % len(cams)]
        params = P.RenderParams(cull=(0, 1, 2)[i % 3], lb_cap=(12 if i % 5 == 4 else 0))
        reqs.append((sg, cam, params))
    return scenes, reqs


def test_served_frames_match_adr_render_alone(P):
    import torch
    scenes, reqs = _requests(P)
    say(f"{len(reqs)} requests over {len(scenes)} scenes, mixed sizes, modes and caps")
    ws = P.Workspace()
    alone = []
    for sg, cam, params in reqs:
        o = outputs(cam)
        P.render(sg, cam, params, ws, **o)
        alone.append(o)
    torch.cuda.synchronize()
    srv = P.Server(n_slots=6, max_batch=16, memory_budget=8 << 30)
    served = [outputs(cam) for _, cam, _ in reqs]
    # twice the set, submitted back to back: later requests arrive while
    # earlier ones run, so frames of different requests share blend launches
    tickets = []
    for rnd in range(2):
        for (sg, cam, params), o in zip(reqs, served if rnd == 0 else [outputs(c) for _, c, _ in reqs]):
            tickets.append((srv.submit(sg, cam, params, **o), o))
    infos = [srv.wait(t) for t, _ in tickets]
    st = srv.stats()
    say(f"batches {st['batches']}, largest {st['max_batch_seen']}, reserved peak {st['reserved_bytes_peak']} B, "
        f"pool {st['pool_bytes']} B")
    for k, ((t, o), info) in enumerate(zip(tickets, infos)):
        ref = alone[k % len(reqs)]
        for key in ("image", "final_t", "l_iter", "l_blend", "load_sums", "load_stats"):
            assert torch.equal(o[key], ref[key]), (k, key)
        assert info["status"] == 0 and info["done_s"] >= info["start_s"] >= info["submit_s"]
    assert st["requests_done"] == len(tickets)
    assert st["max_batch_seen"] > 1, "no blend launch held more than one frame"
    assert st["batches"] < len(tickets)
    srv.close()
    ws.close()


def test_admission_keeps_reservations_within_the_budget(P):
    """With a budget that holds about two of the frames at once, the server
    still finishes every request (one is always admitted) and its peak
    reservation stays within the budget whenever more than one request runs."""
    import torch
    sg = P.Scene.from_synth(scene_clusters(200_000, seed=5))
    cam = camera_orbit(20.0, 15.0, 300.0, 1280, 720)
    params = P.RenderParams()
    ws = P.Workspace()
    ref = outputs(cam)
    n = P.render(sg, cam, params, ws, **ref)
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    one = P.Workspace.bytes_for(sg.n, n + n // 4, tiles)
    budget = int(2.5 * one)
    srv = P.Server(n_slots=8, max_batch=8, memory_budget=budget)
    # the first request's estimate (4 N pairs) is not this frame's: warm it up
    srv.wait(srv.submit(sg, cam, params, **outputs(cam)))
    outs = [outputs(cam) for _ in range(12)]
    tickets = [srv.submit(sg, cam, params, **o) for o in outs]
    infos = [srv.wait(t) for t in tickets]
    st = srv.stats()
    say(f"budget {budget} B (one frame {one} B): reserved peak {st['reserved_bytes_peak']} B, "
        f"footprints {sorted(set(i['footprint'] for i in infos))}")
    assert st["reserved_bytes_peak"] <= budget
    for o in outs:
        assert torch.equal(o["image"], ref["image"])
    srv.close()
    ws.close()
