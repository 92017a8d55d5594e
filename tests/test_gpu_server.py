"""Serving (resident scenes, concurrent requests through adr_server): every
frame of a mixed stream of requests must be bitwise the frame adr_render
gives for the same request alone. Runs on an MI355X only."""
import numpy as np
import pytest

from synth import scene_small, scene_clusters, camera_small, camera_orbit

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="serving is switched off: its first GPU run ended in a GPU memory fault "
                                      "whose cause is not found yet; adr_server_create reports ADR_E_UNSUPPORTED")]


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
                load_sums=torch.zeros(4, dtype=torch.int64, device=device))


def test_served_frames_match_adr_render_alone(P):
    import torch
    scenes = [P.Scene.from_synth(scene_small(2000, seed=0)), P.Scene.from_synth(scene_clusters(40_000, seed=3))]
    cams = [camera_small(128, 128), camera_small(130, 70), camera_orbit(30.0, 20.0, 45.0, 320, 240),
            camera_orbit(30.0, 35.0, 200.0, 640, 360)]
    rng = np.random.default_rng(7)
    reqs = [(int(rng.integers(0, 2)), int(rng.integers(0, 4)), int(rng.integers(0, 3)), int(rng.integers(0, 2)))
            for _ in range(24)]
    server = P.Server(4)
    say(f"{len(reqs)} mixed requests on 4 slots")
    outs, tickets = [], []
    for si, ci, mode, cap in reqs:
        o = outputs(cams[ci])
        params = P.RenderParams(cull=mode, lb_cap=4 if cap else 0)
        tickets.append(server.submit(scenes[si], cams[ci], params, **o))
        outs.append(o)
    infos = [server.wait(t) for t in tickets]
    server.close()
    torch.cuda.synchronize()
    say("each against adr_render alone")
    ws = P.Workspace()
    for (si, ci, mode, cap), o, info in zip(reqs, outs, infos):
        assert info["status"] == 0 and info["submit_s"] <= info["start_s"] <= info["done_s"]
        ref = outputs(cams[ci])
        n_pairs = P.render(scenes[si], cams[ci], P.RenderParams(cull=mode, lb_cap=4 if cap else 0), ws, **ref)
        torch.cuda.synchronize()
        assert info["n_pairs"] == n_pairs
        for k in ("image", "final_t", "l_iter", "l_blend", "load_sums"):
            assert torch.equal(o[k], ref[k]), (k, si, ci, mode, cap)


def test_server_rejects_bad_requests_and_retires_tickets(P):
    """Arguments the host can check are rejected at submission, before
    anything is queued; a ticket retires on its first wait."""
    import torch
    scene = P.Scene.from_synth(scene_small(100, seed=1))
    cam = camera_small(64, 64)
    server = P.Server(1)
    o = outputs(cam)
    with pytest.raises(P.AdrError):
        server.submit(scene, cam, P.RenderParams(alpha_low=0.0), **o)  # rejected before queueing
    t = server.submit(scene, cam, P.RenderParams(), **o)
    info = server.wait(t)
    assert info["status"] == 0
    with pytest.raises(P.AdrError):
        server.wait(t)  # retired ticket
    server.close()
    torch.cuda.synchronize()
