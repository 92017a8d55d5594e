"""Frames/s of the forward rasterizer at 1080p with 1M Gaussians (SH degree 3),
adaptive radius + AABB culling vs the plain 3-sigma radius, on one MI355X.

A step is one whole frame through the C ABI: Preprocess with early culling,
InclusiveSum, DuplicateWithKeys, SortPairs, IdentifyTileRanges and Render with
the per-pixel load counters and their sums (Eq. 13). The scene and camera are
resident in HBM before the timed region. Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s at 1080p/1M Gaussians, adaptive vs 3σ radius; serving p99 ms"
HBM_PEAK_GBS = 8000.0
# FP32 VALU without packed instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# x 2 flops per FMA = 78.6 TFLOP/s (the 157.3 TFLOP/s headline needs packed FP32)
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# Flops of the blend definition (Eq. 2-3): per examined list entry, the offset
# (2), the quadratic form (3 mul + 3 fma = 9), exp (1), clamp (1) and the
# alpha_low test (1); per blended entry, the weight (1), three colour FMAs (6),
# 1 - alpha and the transmittance product (2) and the stop test (1).
FLOPS_PER_EXAMINED = 14
FLOPS_PER_BLENDED = 10


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="measured length of the serving run (0 = skip); 2 s of warm-up come first")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-slots", type=int, default=8, help="requests in flight at once")
    ap.add_argument("--serve-batch", type=int, default=16, help="frames per batched blend launch")
    ap.add_argument("--serve-budget-gib", type=float, default=24.0,
                    help="device memory admitted requests may reserve (GiB)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="host processes of the CPU baseline (0: min(16, CPUs of the host))")
    ap.add_argument("--no-lb", action="store_true",
                    help="skip the load-balancing sweep on the 3M-Gaussian load-imbalanced workload")
    ap.add_argument("--train-iters", type=int, default=600, help="iterations per run of --only train")
    ap.add_argument("--only", choices=["3sigma", "adaptive", "aabb", "aabb_pairs_only", "backward", "train", "lb", "seeds",
                                       "serve"],
                    default=None,
                    help="time one mode only (for profiler runs)")
    ap.add_argument("--no-alpha-sweep", action="store_true",
                    help="skip the alpha_low sweep (frames/s and PSNR at 1, 2, 4, 8 / 255)")
    ap.add_argument("--backward", action="store_true",
                    help="also time the gradients (adr_render_backward on the AABB frame) after the modes; "
                         "off by default, --only backward times them alone")
    ap.add_argument("--no-two-in-flight", action="store_true",
                    help="skip the two-workspace, two-stream throughput figure (profiler runs: its overlapped "
                         "launches would enter the kernel averages)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (scales HBM counters)")
    return ap.parse_args()


def algorithmic_bytes(stage, n, n_vis, n_pairs, n_pix, n_tiles, n_coeff, depth_bits):
    """Bytes the method itself must move per launch of each stage (reads +
    writes), independent of how the kernel caches them."""
    if stage == "preprocess":
        # geometry of every Gaussian (48 B) in, tiles_touched + depth key + id
        # (12 B) out; SH of visible ones in, render record (64 B) + FP64
        # record (32 B) + tile rectangle (8 B) out
        return n * (48 + 12) + n_vis * (12 * n_coeff + 64 + 32 + 8)
    if stage == "inclusive_sum":
        # depth order (4 B) and tiles_touched (4 B) of each visible Gaussian, offset out (4 B)
        return n_vis * 12
    if stage == "duplicate":
        # offsets, order and tile rectangle of each visible Gaussian, tile id + id out per pair
        return n_vis * 16 + n_pairs * 8
    if stage in ("depth_sort", "tile_sort"):
        # LSD radix sort with 8-bit digits: per pass the key is read once for
        # the digit counts, then key and id are read and written once
        n_el, bits = (n, depth_bits) if stage == "depth_sort" else (n_pairs, math.ceil(math.log2(n_tiles)))
        return math.ceil(bits / 8) * n_el * 20
    if stage == "ranges":
        return n_pairs * 8 + n_tiles * 8
    if stage == "render":
        # ids + 64-byte records of every pair, image + T + two counters out
        return n_pairs * (4 + 64) + n_pix * 24
    if stage == "tile_order":
        return n_tiles * (8 + 4)
    if stage == "load_sums":
        return n_tiles * 4 * 32
    return 0


KERNEL_SOURCES = {"render_kernel": ("paper_2409_08669_amd/csrc/render.hip", "paper_2409_08669_amd/csrc/adr_internal.h")}
TRAFFIC_PROFILE = "profiles/hbm_traffic_1M_1080p_aabb.md"


def source_digest(kernel):
    """sha256 over the source files a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE passes,
    scaled by a plain copy) from the committed counter summary of the AABB
    headline frame, or None when the kernel's sources changed since the
    counters were taken (the summary records their digest) or it has no row."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    digest, row = None, None
    for line in open(path):
        if line.startswith(f"Source digest of {kernel}:"):
            digest = line.split("`")[1] if line.count("`") >= 2 else None
        if line.startswith(f"| {kernel} "):
            row = [c.strip() for c in line.strip().strip("|").split("|")]
    if digest != source_digest(kernel) or row is None:
        return None
    return int(round((float(row[-2]) + float(row[-1])) * 1e6))


def main():
    args = parse()
    if args.only == "serve":
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        import paper_2409_08669_amd as P
        P.load()
        print(json.dumps({"mode": "serve", "serving": serve_benchmark(P, args)}), flush=True)
        return
    if args.only == "seeds":
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        import paper_2409_08669_amd as P
        P.load()
        print(json.dumps({"mode": "seeds", "seeds": seed_sweep(P, args)}), flush=True)
        return
    if args.only == "lb":
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        import paper_2409_08669_amd as P
        P.load()
        print(json.dumps({"mode": "lb", "lb": cap_sweep(P, args)}), flush=True)
        return
    if args.only == "train":
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"  # torch takes the device first
        import paper_2409_08669_amd as P
        P.load()
        print(json.dumps({"mode": "train", "train": train_load_balancing(P, args)}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (a multi-GPU split is "
                                   "described, not implemented)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2409_08669_amd as P
    from paper_2409_08669_amd.binding import STAGES
    from synth import scene_clusters, camera_1080p

    log(f"generating scene: {args.n} Gaussians, SH degree 3, seed {args.seed}")
    scene = scene_clusters(args.n, seed=args.seed)
    cam = camera_1080p()
    # The CPU baseline first: its worker processes are forked before this
    # process touches the GPU.
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, cam, args.cpu_workers)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.load()
    sg = P.Scene.from_synth(scene)
    ws = P.Workspace()
    w, h = cam.width, cam.height
    dev = "cuda"
    out = dict(image=torch.empty((3, h, w), device=dev), final_t=torch.empty((h, w), device=dev),
               l_iter=torch.empty((h, w), dtype=torch.int32, device=dev),
               l_blend=torch.empty((h, w), dtype=torch.int32, device=dev),
               load_sums=torch.zeros(4, dtype=torch.int64, device=dev),
               load_stats=torch.zeros(4, dtype=torch.float64, device=dev))
    stream = torch.cuda.current_stream()
    n_tiles = ((w + 15) // 16) * ((h + 15) // 16)

    # name: (cull mode, extra flags). The last one is an ablation: the paper's
    # AABB pair culling alone, without reusing the extent inside Render.
    modes = {"3sigma": (P.ADR_CULL_3SIGMA, 0), "adaptive": (P.ADR_CULL_ADAPTIVE, 0),
             "aabb": (P.ADR_CULL_AABB, 0), "aabb_pairs_only": (P.ADR_CULL_AABB, P.ADR_FLAG_NO_QUAD_CULL)}
    if args.only == "backward":
        modes = {}  # the backward section below runs on its own
    elif args.only:
        modes = {args.only: modes[args.only]}
    results = {}
    images = {}
    for name, (mode, extra) in modes.items():
        params = P.RenderParams(cull=mode, flags=extra)
        timed = P.RenderParams(cull=mode, flags=P.ADR_FLAG_TIMING | extra)
        log(f"mode {name}: warmup {args.warmup}")
        for _ in range(args.warmup):
            P.render(sg, cam, params, ws, **out)
        torch.cuda.synchronize()
        # Throughput: frames back to back, no per-stage events (each event
        # record costs a few microseconds of GPU idle time).
        log(f"mode {name}: timing {args.steps} frames")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            n_pairs = P.render(sg, cam, params, ws, **out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # Stage durations: the same frames again with HIP events around every
        # stage, recorded on the library's stream, read after each frame.
        stage_runs = {s: [] for s in STAGES}
        for _ in range(args.steps):
            P.render(sg, cam, timed, ws, **out)
            for k, v in ws.stage_times().items():
                stage_runs[k].append(v)
        torch.cuda.synchronize()
        counters = ws.counters()
        sums = out["load_sums"].cpu().numpy()
        mean_b, std_b, mean_i, std_i = (float(v) for v in out["load_stats"].cpu().numpy())
        results[name] = dict(
            fps=args.steps / dt, ms_per_frame=1e3 * dt / args.steps, pairs=int(n_pairs),
            sum_blend=int(sums[0]), sum_iter=int(sums[2]),
            visible=counters.get("visible"), depth_bits=counters.get("depth_sort_bits"),
            stages_ms={k: float(np.mean(v)) for k, v in stage_runs.items()},
            stages_ms_pctl={k: [round(float(x), 4) for x in np.percentile(v, [10, 50, 90])]
                            for k, v in stage_runs.items()},
            band_redecisions=counters.get("band_redecisions"), t_replays=counters.get("t_replays"),
            load_mean_blend=mean_b, load_std_blend=std_b, load_mean_iter=mean_i, load_std_iter=std_i)
        images[name] = out["image"].clone()
        results[name]["fps_two_in_flight"] = (None if args.no_two_in_flight else
                                              two_in_flight(P, sg, cam, params, args.steps, args.warmup, out))
        if name == "aabb":
            # Load imbalance of the paper's pixel-parallel blend: every wave
            # (8 x 8 pixels) runs as long as its longest pixel list, so its
            # executed work is 64 x max l_iter against the sum of l_iter.
            li = out["l_iter"].cpu().numpy().astype(np.int64)
            hp, wp = -(-h // 8) * 8, -(-w // 8) * 8
            pad = np.zeros((hp, wp), dtype=np.int64)
            pad[:h, :w] = li
            wave_max = pad.reshape(hp // 8, 8, wp // 8, 8).max(axis=(1, 3))
            results[name]["load_imbalance_E_exec_over_E_alg"] = round(float(64 * wave_max.sum() / max(li.sum(), 1)), 4)
        log(f"mode {name}: {results[name]['fps']:.1f} frames/s, pairs {n_pairs}, stages "
            + ", ".join(f"{k} {v:.3f}" for k, v in results[name]["stages_ms"].items()))
    identical = True
    if images:
        first = next(iter(images.values()))
        identical = all(bool(torch.equal(first, im)) for im in images.values())
    if args.copy_probe_mib:
        n_el = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n_el, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
    # Measured device copy bandwidth (512 MiB read + 512 MiB written per copy),
    # the practical HBM ceiling the stage fractions are also quoted against.
    copy_gbs = None
    if not args.only:
        src = torch.ones(128 << 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
    # alpha_low sweep (a lossy speed-up the paper allows, Sec. 5.1.2): the
    # headline AABB frame at larger alpha_low, with its PSNR against the
    # alpha_low = 1/255 image (both clipped to [0, 1]).
    alpha_sweep = None
    if not args.only and not args.no_alpha_sweep:
        alpha_sweep = []
        ref_img = images["aabb"].clamp(0.0, 1.0)
        for k in (1, 2, 4, 8):
            params = P.RenderParams(cull=P.ADR_CULL_AABB, alpha_low=k / 255.0)
            for _ in range(args.warmup):
                P.render(sg, cam, params, ws, **out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                n_pairs = P.render(sg, cam, params, ws, **out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            mse = float(((out["image"].clamp(0.0, 1.0) - ref_img) ** 2).mean())
            psnr = None if mse == 0.0 else round(10.0 * math.log10(1.0 / mse), 3)
            alpha_sweep.append({"alpha_low": f"{k}/255", "fps": round(args.steps / dt, 2), "pairs": int(n_pairs),
                                "psnr_db_vs_1_255": psnr, "identical_to_1_255": mse == 0.0})
            log(f"alpha_low {k}/255: {args.steps / dt:.1f} frames/s, pairs {n_pairs}, PSNR {psnr}")
    # Gradients (next row 2): adr_render_backward of the AABB frame for a
    # seeded dL/dimage, timed alone (the same forward differentiated again)
    # and as forward + backward back to back.
    backward = None
    if (not args.only and args.backward) or args.only == "backward":
        params = P.RenderParams(cull=P.ADR_CULL_AABB)
        frame = {k: out[k] for k in ("image", "final_t", "l_iter")}
        gen = torch.Generator(device=dev).manual_seed(args.seed)
        dl = torch.randn((3, h, w), device=dev, generator=gen)
        for _ in range(max(args.warmup // 2, 1)):
            P.render(sg, cam, params, ws, **out)
            P.render_backward(sg, cam, params, ws, frame, dl)
        torch.cuda.synchronize()
        nb = max(args.steps // 2, 1)
        t0 = time.perf_counter()
        for _ in range(nb):
            P.render(sg, cam, params, ws, **out)
            g = P.render_backward(sg, cam, params, ws, frame, dl)
        torch.cuda.synchronize()
        fwd_bwd = (time.perf_counter() - t0) / nb
        t0 = time.perf_counter()
        for _ in range(nb):
            g = P.render_backward(sg, cam, params, ws, frame, dl)
        torch.cuda.synchronize()
        bwd = (time.perf_counter() - t0) / nb
        backward = {"ms_backward": round(bwd * 1e3, 4), "ms_forward_plus_backward": round(fwd_bwd * 1e3, 4),
                    "frames_per_s_forward_plus_backward": round(1.0 / fwd_bwd, 2),
                    "grad_abs_max": {k: float(v.abs().max()) for k, v in g.items()}}
        log(f"backward: {bwd * 1e3:.3f} ms alone, forward + backward {fwd_bwd * 1e3:.3f} ms")
    if args.only == "backward":
        print(json.dumps({"mode": "backward", "backward": backward}), flush=True)
        return
    if args.only:
        r = results[args.only]
        print(json.dumps({"mode": args.only, "fps": round(r["fps"], 2), "pairs": r["pairs"],
                          "stages_ms": {k: round(v, 4) for k, v in r["stages_ms"].items()}}), flush=True)
        return

    # Roofline of the dominant kernel of the headline (AABB) frame. The blend
    # kernel is bound by FP32 VALU work: its algorithmic work is the paper's
    # pixel-parallel cost, sum over pixels of the list entries examined
    # (l_iter) and blended (l_blend), both exact from the frame's load sums.
    head = results["aabb"]
    n_vis = head["visible"] or args.n
    kern = {k: v for k, v in head["stages_ms"].items() if k != "host_wait"}
    dom = max(kern, key=kern.get)
    per_stage = {}
    for s_, ms in kern.items():
        b = algorithmic_bytes(s_, args.n, n_vis, head["pairs"], w * h, n_tiles, 16, head["depth_bits"] or 32)
        per_stage[s_] = {"ms": round(ms, 4), "algorithmic_bytes": int(b),
                         "GB/s": round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                         "frac_hbm": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None,
                         "frac_copy": round(b / (ms * 1e-3) / 1e9 / copy_gbs, 4) if ms > 0 and copy_gbs else None,
                         "ms_p10_p50_p90": head["stages_ms_pctl"][s_]}
    if dom == "render":
        flops = FLOPS_PER_EXAMINED * head["sum_iter"] + FLOPS_PER_BLENDED * head["sum_blend"]
        achieved = flops / (kern[dom] * 1e-3) / 1e12
        roofline = {"kernel": "render_kernel", "bound": "alu", "achieved": round(achieved, 3),
                    "peak": round(VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                    "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": measured_traffic("render_kernel"),
                    "algorithmic_flops": int(flops), "examined": head["sum_iter"], "blended": head["sum_blend"],
                    "avg_ms": round(kern[dom], 4)}
    else:
        b = per_stage[dom]["algorithmic_bytes"]
        achieved = b / (kern[dom] * 1e-3) / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "algorithmic_bytes": int(b), "avg_ms": round(kern[dom], 4)}

    lb = None
    if not args.no_lb:
        del ws
        lb = cap_sweep(P, args)
    serving = None
    if args.serve_seconds > 0:
        del sg, out, images
        torch.cuda.empty_cache()
        serving = serve_benchmark(P, args)

    line = {
        "metric": METRIC,
        "value": round(head["fps"], 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_frame"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M Gaussians (64-cluster mixture, SH degree 3), one 1920x1080 orbit camera, "
                               "adaptive-radius+AABB culling (3-sigma and adaptive also timed)",
                   "n_gaussians": args.n, "width": w, "height": h, "sh_degree": 3, "cull": "aabb",
                   "alpha_low": 1.0 / 255.0, "seed": args.seed},
        "modes": {k: {"fps": round(v["fps"], 2), "ms_per_frame": round(v["ms_per_frame"], 4),
                      "fps_two_in_flight": (round(v["fps_two_in_flight"], 2) if v["fps_two_in_flight"] else None),
                      "pairs_per_frame": v["pairs"], "stages_ms": {s_: round(x, 4) for s_, x in v["stages_ms"].items()},
                      "load_std_blend": round(v["load_std_blend"], 4), "load_std_iter": round(v["load_std_iter"], 4),
                      "band_redecisions": v["band_redecisions"], "t_replays": v["t_replays"]}
                  for k, v in results.items()},
        "speedup_aabb_vs_3sigma": round(results["aabb"]["fps"] / results["3sigma"]["fps"], 4),
        "speedup_adaptive_vs_3sigma": round(results["adaptive"]["fps"] / results["3sigma"]["fps"], 4),
        "identical_output_across_modes": identical,
        "alpha_low_sweep": alpha_sweep,
        "backward": backward,
        "stages": per_stage,
        "hbm_copy_GBs": round(copy_gbs, 1) if copy_gbs else None,
        "load_imbalance_E_exec_over_E_alg": results["aabb"].get("load_imbalance_E_exec_over_E_alg"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "load_balancing": lb,
        "serving_p99_ms": serving["p99_ms"] if serving else None,
        "serving": serving,
        "paper_context": "paper reports ~3.1x over 3DGS (Ours-Full, RTX 3090, trained scenes); AABB alone 1.65-2.11x",
    }
    print(json.dumps(line), flush=True)


def two_in_flight(P, sg, cam, params, steps, warmup, like):
    """Frames/s with consecutive frames alternating between two workspaces on
    two streams (default priority) and two sets of outputs, so that the blends
    of consecutive frames may overlap too (on one workspace and one set of
    outputs they are ordered on the caller's stream). Every frame is still
    whole; only their overlap differs from the back-to-back figure."""
    import torch
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    spaces = [P.Workspace(), P.Workspace()]
    outs = [{k: torch.empty_like(v) for k, v in like.items()} for _ in range(2)]
    torch.cuda.synchronize()
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        k = i % 2
        P.render(sg, cam, params, spaces[k], **outs[k], stream=streams[k].cuda_stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for w in spaces:
        w.close()
    return steps / dt


def _ssim(img, ref):
    """Mean SSIM of two (3, H, W) images: 11 x 11 Gaussian window, sigma 1.5,
    C1 = 0.01^2, C2 = 0.03^2 (the usual constants for [0, 1] images)."""
    import torch
    import torch.nn.functional as F
    x = torch.arange(11, dtype=img.dtype, device=img.device) - 5.0
    g = torch.exp(-x * x / (2 * 1.5 ** 2))
    g = g / g.sum()
    win = (g[:, None] * g[None, :]).expand(3, 1, 11, 11).contiguous()
    a, b = img[None], ref[None]
    mu_a = F.conv2d(a, win, padding=5, groups=3)
    mu_b = F.conv2d(b, win, padding=5, groups=3)
    s_aa = F.conv2d(a * a, win, padding=5, groups=3) - mu_a * mu_a
    s_bb = F.conv2d(b * b, win, padding=5, groups=3) - mu_b * mu_b
    s_ab = F.conv2d(a * b, win, padding=5, groups=3) - mu_a * mu_b
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    m = ((2 * mu_a * mu_b + c1) * (2 * s_ab + c2)) / ((mu_a * mu_a + mu_b * mu_b + c1) * (s_aa + s_bb + c2))
    return m.mean()


def seed_sweep(P, args):
    """The headline workload (1M Gaussians, SH3, 1920x1080 orbit camera) for
    scene seeds 0, 1 and 2: frames/s (back-to-back frames after warm-up),
    pairs per frame, list entries examined and blended (the load sums) and the
    blend's FP64 fallbacks of the three cull modes, and whether their images
    are bitwise identical."""
    import numpy as np
    import torch
    from synth import scene_clusters, camera_1080p

    cam = camera_1080p()
    w, h = cam.width, cam.height
    dev = "cuda"
    out = dict(image=torch.empty((3, h, w), device=dev), final_t=torch.empty((h, w), device=dev),
               l_iter=torch.empty((h, w), dtype=torch.int32, device=dev),
               l_blend=torch.empty((h, w), dtype=torch.int32, device=dev),
               load_sums=torch.zeros(4, dtype=torch.int64, device=dev),
               load_stats=torch.zeros(4, dtype=torch.float64, device=dev))
    ws = P.Workspace()
    res = []
    for seed in (0, 1, 2):
        log(f"seed sweep: scene seed {seed}")
        sg = P.Scene.from_synth(scene_clusters(args.n, seed=seed))
        row = {"seed": seed}
        images = []
        for name, mode in (("3sigma", P.ADR_CULL_3SIGMA), ("adaptive", P.ADR_CULL_ADAPTIVE), ("aabb", P.ADR_CULL_AABB)):
            params = P.RenderParams(cull=mode)
            for _ in range(args.warmup):
                P.render(sg, cam, params, ws, **out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                n_pairs = P.render(sg, cam, params, ws, **out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            sums = out["load_sums"].cpu().numpy()
            cnt = ws.counters()
            row[name] = {"fps": round(1.0 / dt, 2), "pairs": int(n_pairs), "examined": int(sums[2]),
                         "blended": int(sums[0]), "t_replays": cnt.get("t_replays"),
                         "band_redecisions": cnt.get("band_redecisions")}
            if name == "aabb":  # load imbalance E_exec / E_alg of the 8 x 8 pixel waves
                li = out["l_iter"].cpu().numpy().astype(np.int64)
                hp, wp = -(-h // 8) * 8, -(-w // 8) * 8
                pad = np.zeros((hp, wp), dtype=np.int64)
                pad[:h, :w] = li
                wave_max = pad.reshape(hp // 8, 8, wp // 8, 8).max(axis=(1, 3))
                row[name]["E_exec_over_E_alg"] = round(float(64 * wave_max.sum() / max(li.sum(), 1)), 4)
                row[name]["heaviest_wave_examined"] = int(wave_max.max())
            images.append(out["image"].clone())
        row["identical_images"] = all(bool(torch.equal(images[0], im)) for im in images[1:])
        row["speedup_aabb_vs_3sigma"] = round(row["aabb"]["fps"] / row["3sigma"]["fps"], 4)
        res.append(row)
        log(f"seed {seed}: " + ", ".join(f"{k} {row[k]['fps']:.1f} frames/s {row[k]['pairs']} pairs"
                                        for k in ("3sigma", "adaptive", "aabb")) + f", identical {row['identical_images']}")
        del sg
    return res


def cap_sweep(P, args):
    """The load-balancing mode (a render-time cap of K blends per pixel, the
    reading of Sec. 4.4's compression of heavy-load pixels) on the
    load-imbalanced workload: 3M Gaussians with 20% in 8 dense clusters,
    1600x1040, the 32 poses of the orbit sweep. K = ceil(mean + kappa std) of
    l_blend over the covered pixels of pose 0's exact AABB frame, kappa = 1, 2,
    3. Per pose, exact AABB and each cap: frames/s (back-to-back frames),
    std(l_blend) over all pixels (Eq. 13, from the exact integer sums), and the
    PSNR of the capped image against the exact one (both clipped to [0, 1])."""
    import numpy as np
    import torch
    from synth import scene_heavy, cameras_sweep

    log("cap sweep: 3M-Gaussian load-imbalanced scene, 32 poses at 1600x1040")
    scene = scene_heavy(3_000_000, seed=args.seed)
    sg = P.Scene.from_synth(scene)
    cams = cameras_sweep(32)
    ws = P.Workspace()
    w, h = cams[0].width, cams[0].height
    dev = "cuda"
    out = dict(image=torch.empty((3, h, w), device=dev), final_t=torch.empty((h, w), device=dev),
               l_iter=torch.empty((h, w), dtype=torch.int32, device=dev),
               l_blend=torch.empty((h, w), dtype=torch.int32, device=dev),
               load_sums=torch.zeros(4, dtype=torch.int64, device=dev),
               load_stats=torch.zeros(4, dtype=torch.float64, device=dev))
    exact = P.RenderParams(cull=P.ADR_CULL_AABB)
    P.render(sg, cams[0], exact, ws, **out)
    lb = out["l_blend"][out["l_blend"] > 0].double()
    lb_mean, lb_std = float(lb.mean()), float(lb.std(unbiased=False))
    caps = {k: int(math.ceil(lb_mean + k * lb_std)) for k in (1, 2, 3)}
    log(f"cap sweep: pose 0 covered-pixel l_blend mean {lb_mean:.2f} std {lb_std:.2f}, K {caps}")
    n_rep = max(args.steps // 5, 3)

    def run(cam, params):
        for _ in range(2):
            P.render(sg, cam, params, ws, **out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_rep):
            P.render(sg, cam, params, ws, **out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_rep
        std_b = float(out["load_stats"][1])
        return 1.0 / dt, std_b, out["image"].clamp(0.0, 1.0).clone()

    rows = []
    for pi, cam in enumerate(cams):
        fps_e, std_e, img_e = run(cam, exact)
        row = {"pose": pi, "exact": {"fps": round(fps_e, 2), "std_blend": round(std_e, 3)}}
        for k, cap in caps.items():
            fps_c, std_c, img_c = run(cam, P.RenderParams(cull=P.ADR_CULL_AABB, lb_cap=cap))
            mse = float(((img_c - img_e) ** 2).mean())
            row[f"kappa{k}"] = {"fps": round(fps_c, 2), "std_blend": round(std_c, 3),
                                "psnr_db": None if mse == 0.0 else round(10.0 * math.log10(1.0 / mse), 3)}
        rows.append(row)
        log(f"cap sweep pose {pi}: exact {fps_e:.1f} frames/s std {std_e:.2f}; "
            + "; ".join(f"k{k} {row[f'kappa{k}']['fps']:.1f} fps std {row[f'kappa{k}']['std_blend']:.2f} "
                        f"PSNR {row[f'kappa{k}']['psnr_db']}" for k in caps))
    mean = {"exact": {"fps": round(float(np.mean([r["exact"]["fps"] for r in rows])), 2),
                      "std_blend": round(float(np.mean([r["exact"]["std_blend"] for r in rows])), 3)}}
    for k in caps:
        ps = [r[f"kappa{k}"]["psnr_db"] for r in rows if r[f"kappa{k}"]["psnr_db"] is not None]
        mean[f"kappa{k}"] = {"K": caps[k],
                             "fps": round(float(np.mean([r[f"kappa{k}"]["fps"] for r in rows])), 2),
                             "std_blend": round(float(np.mean([r[f"kappa{k}"]["std_blend"] for r in rows])), 3),
                             "psnr_db": round(float(np.mean(ps)), 3) if ps else None}
    oracle_check = cap_oracle_check(P, scene, sg, cams[0], caps, ws, out)
    return {"n_gaussians": 3_000_000, "width": w, "height": h, "poses": len(cams), "frames_per_setting": n_rep,
            "pose0_covered_lblend_mean": round(lb_mean, 3), "pose0_covered_lblend_std": round(lb_std, 3),
            "caps": caps, "mean": mean, "oracle_check_pose0": oracle_check, "per_pose": rows}


def cap_oracle_check(P, scene, sg, cam, caps, ws, out, n_tiles_sample=16):
    """Pose 0 of the load-balancing sweep against the FP64 oracle on seeded
    tiles: for the exact frame and each cap K, the largest per-channel
    difference from the oracle run with the same K (the parity bar is 2e-4),
    and the PSNR of the capped GPU image against the exact oracle image on
    those tiles (both clipped to [0, 1])."""
    import numpy as np
    import oracle as O

    log(f"cap sweep: oracle check of pose 0 on {n_tiles_sample} seeded tiles")
    params = O.Params(cull=O.CULL_AABB)
    pre = O.preprocess(scene, cam, params)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    tx, ty = O.n_tiles(cam)
    tiles = np.random.default_rng(17).choice(tx * ty, n_tiles_sample, replace=False)
    ref = O.render_image(pre, values, ranges, cam, params, tiles=tiles)
    mask = ref["done"]
    ref_img = np.clip(ref["image"][:, mask], 0.0, 1.0)
    res = {"tiles": int(tiles.size), "pixels": int(mask.sum())}
    for name, k in [("exact", 0)] + [(f"kappa{kk}", caps[kk]) for kk in sorted(caps)]:
        P.render(sg, cam, P.RenderParams(cull=P.ADR_CULL_AABB, lb_cap=k), ws, **out)
        g = out["image"].cpu().numpy()[:, mask]
        o = ref if k == 0 else O.render_image(pre, values, ranges, cam, O.Params(cull=O.CULL_AABB, lb_cap=k),
                                              tiles=tiles)
        mse = float(np.mean((np.clip(g, 0.0, 1.0) - ref_img) ** 2))
        res[name] = {"K": k, "max_abs_diff_vs_same_K_oracle": float(np.abs(g - o["image"][:, mask]).max()),
                     "psnr_db_vs_exact_oracle": None if mse == 0.0 else round(10.0 * math.log10(1.0 / mse), 3)}
    return res


def train_load_balancing(P, args):
    """The load-balancing loss as training (Eqs. 12-14): starting from a
    synthetic scene, fit its own renders from 16 orbit views with
    L = l1 L1 + ls (1 - SSIM) + ll std(l_blend) for ll = 0.45 (the paper's
    weight), 0.1, 0.02 and 0 (control), (l1, ls) = (0.8, 0.2) (1 - ll) (the
    3DGS split of what the load weight leaves). The load's gradient reaches the Gaussians through
    adr_render_backward_load (slope 1 per blended alpha). Adam with the 3DGS
    learning rates. Reports, per run, PSNR against the targets, the std of the
    per-pixel load and frames/s over the views, before and after."""
    import numpy as np
    import torch
    from synth import scene_clusters, camera_orbit
    torch.manual_seed(args.seed)
    n, w, h, views = 200_000, 480, 272, 16
    gt = scene_clusters(n, seed=args.seed + 7, sh_degree=0)
    cams = [camera_orbit(30.0, 20.0, 360.0 * k / views, w, h, 60.0) for k in range(views)]
    prm = P.RenderParams(cull=P.ADR_CULL_AABB)
    ws = P.Workspace()
    dev = "cuda"

    def frame():
        return dict(image=torch.empty((3, h, w), device=dev), final_t=torch.empty((h, w), device=dev),
                    l_iter=torch.empty((h, w), dtype=torch.int32, device=dev),
                    l_blend=torch.empty((h, w), dtype=torch.int32, device=dev))

    def evaluate(scene, targets=None):
        imgs, stds = [], []
        for cam in cams:
            f = frame()
            P.render(scene, cam, prm, ws, **f)
            imgs.append(f["image"].clone())
            stds.append(float(f["l_blend"].float().std(unbiased=False)))
        torch.cuda.synchronize()
        for cam in cams:  # warm
            P.render(scene, cam, prm, ws, **f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            for cam in cams:
                P.render(scene, cam, prm, ws, **f)
        torch.cuda.synchronize()
        fps = 5 * len(cams) / (time.perf_counter() - t0)
        psnr = None
        if targets is not None:
            mse = float(torch.stack([((a.clamp(0, 1) - b.clamp(0, 1)) ** 2).mean() for a, b in zip(imgs, targets)]).mean())
            psnr = None if mse == 0.0 else 10.0 * math.log10(1.0 / mse)
        return imgs, float(np.mean(stds)), fps, psnr

    gt_scene = P.Scene.from_synth(gt)
    targets, std_gt, fps_gt, _ = evaluate(gt_scene)
    log(f"train: {n} Gaussians, {views} views at {w}x{h}; targets std(l_blend) {std_gt:.2f}, {fps_gt:.0f} frames/s")
    runs = []
    for ll in (0.45, 0.1, 0.02, 0.0):
        l1, ls = 0.8 * (1.0 - ll), 0.2 * (1.0 - ll)  # the weights sum to 1 (Eq. 14)
        t = {k: torch.tensor(np.asarray(getattr(gt, k), dtype=np.float32), device=dev)
             for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
        lrs = {"means": 1.6e-4 * 10.0, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
        opt = torch.optim.Adam([{"params": [t[k]], "lr": lrs[k]} for k in t], eps=1e-15)
        t0 = time.perf_counter()
        for it in range(args.train_iters):
            cam = cams[it % views]
            scene = P.Scene(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], 0)
            f = frame()
            P.render(scene, cam, prm, ws, **f)
            img = f["image"].detach().requires_grad_(True)
            loss_img = l1 * (img - targets[it % views]).abs().mean() + ls * (1.0 - _ssim(img, targets[it % views]))
            loss_img.backward()
            dload = None
            if ll > 0:
                lb = f["l_blend"].float()
                sd = lb.std(unbiased=False)
                if float(sd) > 0:
                    dload = ll * (lb - lb.mean()) / (lb.numel() * sd)  # d std / d l_i, Eq. 13
            g = P.render_backward(scene, cam, prm, ws, f, img.grad, dl_dload=dload)
            for k in t:
                t[k].grad = g[k]
            opt.step()
            opt.zero_grad(set_to_none=True)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        scene = P.Scene(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], 0)
        _, std_after, fps_after, psnr = evaluate(scene, targets)
        runs.append({"lambda_l1": l1, "lambda_ssim": ls, "lambda_load": ll, "iters": args.train_iters,
                     "train_s": round(secs, 2), "psnr_db_vs_targets": None if psnr is None else round(psnr, 3),
                     "load_std_before": round(std_gt, 3), "load_std_after": round(std_after, 3),
                     "fps_before": round(fps_gt, 1), "fps_after": round(fps_after, 1)})
        log(f"train lambda_load {ll}: std(l_blend) {std_gt:.2f} -> {std_after:.2f}, "
            f"{fps_gt:.0f} -> {fps_after:.0f} frames/s, PSNR {psnr}")
    return {"gaussians": n, "views": views, "width": w, "height": h, "cull": "aabb", "runs": runs}


def serve_benchmark(P, args):
    """Serving load: resident scenes of 0.5, 1, 2 and 3M Gaussians (the
    headline generator, seeds 1..4), Poisson arrivals at args.serve_rate
    requests/s, each request a uniformly drawn scene and resolution (640x480,
    1280x720, 1920x1080, 3840x2160) and an orbit pose (azimuth U[0, 360),
    elevation U[5, 45] degrees, radius 30), AABB culling. Latency = arrival
    (the scheduled time, on the server's clock) to the frame's completion on
    the device; 2 s of warm-up arrivals are not counted."""
    import threading
    import numpy as np
    import torch
    from synth import scene_clusters, camera_orbit

    sizes = (500_000, 1_000_000, 2_000_000, 3_000_000)
    res = ((640, 480), (1280, 720), (1920, 1080), (3840, 2160))
    log(f"serving: generating {len(sizes)} resident scenes")
    scenes = [P.Scene.from_synth(scene_clusters(n, seed=1 + i)) for i, n in enumerate(sizes)]
    rng = np.random.default_rng(2024)
    warm, total = 2.0, 2.0 + args.serve_seconds
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / args.serve_rate)
        if t >= total:
            break
        w, h = res[rng.integers(0, len(res))]
        cam = camera_orbit(30.0, rng.uniform(5.0, 45.0), rng.uniform(0.0, 360.0), int(w), int(h))
        arrivals.append((t, int(rng.integers(0, len(scenes))), cam))
    # output buffers: a pool sized for the largest frame, recycled once a
    # request completes (waiting for a free one counts toward latency)
    n_buf = 32
    wmax, hmax = res[-1]
    pool = [dict(image=torch.empty((3, hmax, wmax), device="cuda")) for _ in range(n_buf)]
    free = list(range(n_buf))
    cv = threading.Condition()
    budget = int(args.serve_budget_gib * (1 << 30))
    server = P.Server(n_slots=args.serve_slots, max_batch=args.serve_batch, memory_budget=budget)
    params = P.RenderParams(cull=P.ADR_CULL_AABB)
    pending, done = [], []

    def collect():
        while True:
            with cv:
                while not pending:
                    cv.wait()
                item = pending.pop(0)
            if item is None:
                return
            arrival, ticket, b, sc, cam = item
            info = server.wait(ticket)
            with cv:
                free.append(b)
                done.append((arrival, info, sc, cam.width * cam.height))
                cv.notify_all()

    th = threading.Thread(target=collect)
    th.start()
    log(f"serving: {len(arrivals)} requests over {total:.0f} s at {args.serve_rate:.0f}/s on {args.serve_slots} slots")
    t0 = P.clock_s() + 0.2
    for t_arr, sc, cam in arrivals:
        arrival = t0 + t_arr
        while P.clock_s() < arrival:
            time.sleep(max(0.0, min(arrival - P.clock_s() - 2e-4, 1e-3)))
        with cv:
            while not free:
                cv.wait()
            b = free.pop()
        img = pool[b]["image"]
        view = img.view(-1)[: 3 * cam.height * cam.width].view(3, cam.height, cam.width)
        ticket = server.submit(scenes[sc], cam, params, view, arrival_s=arrival)
        with cv:
            pending.append((arrival, ticket, b, sc, cam))
            cv.notify_all()
    with cv:
        pending.append(None)
        cv.notify_all()
    th.join()
    st = server.stats()
    server.close()
    lat = np.array([(info["done_s"] - arr) * 1e3 for arr, info, _, _ in done if arr - t0 >= warm])
    batch_sizes = np.array([info["batch_size"] for arr, info, _, _ in done if arr - t0 >= warm])
    queue_ms = np.array([(info["start_s"] - arr) * 1e3 for arr, info, _, _ in done if arr - t0 >= warm])
    span = max(info["done_s"] for _, info, _, _ in done) - (t0 + warm)
    by_res = {}
    for arr, info, sc, px in done:
        if arr - t0 >= warm:
            by_res.setdefault(px, []).append((info["done_s"] - arr) * 1e3)
    names = {w * h: f"{w}x{h}" for w, h in res}
    return {"rate_per_s": args.serve_rate, "seconds": args.serve_seconds, "slots": args.serve_slots,
            "max_batch": args.serve_batch, "memory_budget_bytes": budget,
            "batches": int(st["batches"]), "largest_batch": int(st["max_batch_seen"]),
            "mean_frames_per_blend_launch": round(float(batch_sizes.mean()), 3),
            "reserved_bytes_peak": int(st["reserved_bytes_peak"]), "pool_bytes": int(st["pool_bytes"]),
            "admission_wait_p99_ms": round(float(np.percentile(queue_ms, 99)), 3),
            "requests": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "max_ms": round(float(lat.max()), 3),
            "frames_per_s": round(lat.size / span, 1),
            "p50_ms_by_resolution": {names[k]: round(float(np.percentile(v, 50)), 3) for k, v in sorted(by_res.items())},
            "p99_ms_by_resolution": {names[k]: round(float(np.percentile(v, 99)), 3) for k, v in sorted(by_res.items())},
            "scenes": list(sizes), "cull": "aabb",
            "workload": "Poisson arrivals; scene uniform over the resident scenes; resolution uniform over "
                        "640x480, 1280x720, 1920x1080, 3840x2160; orbit pose radius 30, elevation U[5,45], "
                        "azimuth U[0,360)"}


_CPU_STATE = {}


def _cpu_tiles(tiles):
    """Worker: the oracle's blend of a list of tiles (forked: reads the
    frame's Preprocess and pair lists from the parent's memory)."""
    import oracle as O
    st = _CPU_STATE
    t0 = time.perf_counter()
    O.render_image(st["pre"], st["values"], st["ranges"], st["cam"], st["params"], tiles=tiles)
    return time.perf_counter() - t0


def _oracle_frame_parallel(scene, cam, params, workers):
    """One full frame of the FP64 oracle: Preprocess, emission and sort in
    this process (NumPy, one thread), then the blend of every tile spread over
    `workers` forked processes (tile rows interleaved so that each worker
    gets a mix of heavy and light tiles). Returns (seconds, setup seconds)."""
    import multiprocessing as mp
    import numpy as np

    import oracle as O
    t0 = time.perf_counter()
    pre = O.preprocess(scene, cam, params)
    rects = O.tile_rects(pre, cam, params)
    keys, values, _ = O.duplicate_and_sort(pre, rects, cam)
    ranges = O.tile_ranges(keys, cam)
    t1 = time.perf_counter()
    _CPU_STATE.update(pre=pre, values=values, ranges=ranges, cam=cam, params=params)
    tx, ty = O.n_tiles(cam)
    order = np.argsort(-(ranges[:, 1].astype(np.int64) - ranges[:, 0]), kind="stable")  # longest first
    chunks = [order[i::workers * 4].tolist() for i in range(workers * 4)]
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_cpu_tiles, chunks, chunksize=1)
    t2 = time.perf_counter()
    _CPU_STATE.clear()
    return t2 - t0, t1 - t0


def cpu_baseline(scene, cam, workers):
    """The FP64 oracle timed on the host's cores: the whole headline frame
    (AABB culling; every tile blended, nothing extrapolated), and the small
    parity frame in the three cull modes. Runs before this process touches
    the GPU, so the forked workers never hold GPU state."""
    import oracle as O
    from synth import scene_small, camera_small

    workers = workers or min(16, os.cpu_count() or 1)
    log(f"cpu baseline: FP64 oracle, whole 1080p frame, {workers} processes")
    sec, setup = _oracle_frame_parallel(scene, cam, O.Params(cull=O.CULL_AABB), workers)
    small = {}
    s1, c1 = scene_small(2000, seed=0), camera_small()
    for name, mode in (("3sigma", O.CULL_3SIGMA), ("adaptive", O.CULL_ADAPTIVE), ("aabb", O.CULL_AABB)):
        t, _ = _oracle_frame_parallel(s1, c1, O.Params(cull=mode), workers)
        small[name] = round(1.0 / t, 3)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    log(f"cpu baseline: {sec:.2f} s per frame ({setup:.2f} s Preprocess + sort in one process)")
    return {"value": round(1.0 / sec, 5), "unit": "frames/s", "cores": workers, "kind": "oracle",
            "seconds_per_frame": round(sec, 3),
            "sample": f"one whole frame of the headline workload (1M Gaussians, SH3, 1920x1080, AABB): FP64 "
                      f"NumPy oracle, Preprocess + emission + sort in one process ({setup:.1f} s), the blend of "
                      f"all tiles over {workers} forked processes; nothing extrapolated",
            "small_frame_fps": {"workload": "2000 Gaussians, SH0, 128x128", **small},
            "host_cpus": os.cpu_count(), "cpu_model": model}


if __name__ == "__main__":
    main()
