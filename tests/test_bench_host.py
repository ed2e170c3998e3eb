"""bench.py host logic (no GPU): the multi-GPU refusal and the rule that the
HBM traffic figure is reported only for the workload, tile shape and kernel
sources its counter summary was taken with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _summary(path, workload, digest, traffic=123456):
    with open(path, "w") as f:
        f.write("# counters\n\n```\n")
        f.write("kernel: k_train_raster<16,16,128,1>\n")
        f.write(f"workload: {workload}\n")
        f.write("kernel_sources: paper_2501_08174_amd/csrc/raster.hip paper_2501_08174_amd/csrc/common.h "
                "paper_2501_08174_amd/csrc/launch.h\n")
        f.write(f"kernel_source_sha256: {digest}\n")
        f.write(f"traffic_bytes_per_launch: {traffic}\n```\n")


def _digest():
    import hashlib
    h = hashlib.sha256()
    for rel in ("paper_2501_08174_amd/csrc/raster.hip", "paper_2501_08174_amd/csrc/common.h",
                "paper_2501_08174_amd/csrc/launch.h"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def test_traffic_only_for_matching_workload_tile_and_sources(tmp_path, monkeypatch):
    p = str(tmp_path / "traffic.md")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", p)
    _summary(p, "ragged16-1m 16x16", _digest())
    assert bench.measured_traffic("ragged16-1m", (16, 16)) == 123456
    assert bench.measured_traffic("ragged16-1m", (16, 8)) is None
    assert bench.measured_traffic("wide8-3m", (16, 16)) is None
    _summary(p, "ragged16-1m 16x16", "0" * 64)          # sources changed since the counters
    assert bench.measured_traffic("ragged16-1m", (16, 16)) is None
    os.remove(p)
    assert bench.measured_traffic("ragged16-1m", (16, 16)) is None

