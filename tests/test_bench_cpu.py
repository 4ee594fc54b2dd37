"""Host-side checks of bench.py that need no GPU: it measures one GPU only,
and the counter-derived figures of its JSON line (HBM traffic, VALU
instructions per visit) are reported only for the kernel source they were
counted on."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1608_05238_amd", "csrc", "mcrad.hip")


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_figures_follow_the_kernel_source(monkeypatch):
    import bench
    with open(SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    t = dict(bench.TRAFFIC)
    monkeypatch.setattr(bench, "TRAFFIC", {**t, "source_sha256": sha})
    got = bench.traffic_bytes_per_launch()
    want = 1024.0 * (t["fetch_kib_per_launch"] * t["fetch_factor"] + t["write_kib_per_launch"] * t["write_factor"])
    assert got == want and got > 0
    assert bench.valu_per_visit() == t["valu_per_visit"] > 0
    # another source: the figures no longer describe it
    monkeypatch.setattr(bench, "TRAFFIC", {**t, "source_sha256": "0" * 64})
    assert bench.traffic_bytes_per_launch() is None
    assert bench.valu_per_visit() is None
