"""bench.py on the host: more than one GPU is refused with a message (the
library runs on one GPU), the timing modes are listed, and the roofline's
HBM traffic is read from the committed counter summary only while the
kernel's sources still match the digest recorded there."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_help_lists_the_timing_modes():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for mode in ("aabb", "backward", "train", "lb", "seeds", "serve"):
        assert mode in r.stdout


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_comes_from_the_summary_only_while_the_sources_match(tmp_path, monkeypatch):
    bench = _bench_module()
    digest = bench.source_digest("render_kernel")
    summary = tmp_path / "traffic.md"
    summary.write_text(
        f"Source digest of render_kernel: `{digest}` (sha256 of its sources)\n\n"
        "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB (scaled) | written MB (scaled) |\n"
        "|---|---:|---:|---:|---:|---:|\n"
        "| render_kernel (grid 2088960) | 5 | 221240.7 | 81000.1 | 453.05 | 82.94 |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", "traffic.md")
    monkeypatch.setattr(bench, "source_digest", lambda kernel: digest)
    assert bench.measured_traffic("render_kernel") == 535_990_000  # (453.05 + 82.94) MB
    assert bench.measured_traffic("preprocess_kernel") is None  # no digest kept for it
    monkeypatch.setattr(bench, "source_digest", lambda kernel: "0" * 64)  # the sources changed since
    assert bench.measured_traffic("render_kernel") is None

