"""Host logic of bench.py (no GPU): the one-GPU contract, the roofline arithmetic
and the rule that measured traffic is reported only for the sources it was
measured on."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


class _FakeStats:
    """The fields roofline() reads from alae.Stats."""

    def __init__(self, lane_ms, launches, occ_reads, frontier_bytes):
        self.level_lane_ms = lane_ms
        self.level_lane_launches = launches
        self.occ_reads = occ_reads
        self.frontier_bytes = frontier_bytes

    def level_alg_bytes(self):
        return 64 * self.occ_reads + self.frontier_bytes


def test_roofline_arithmetic(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda workload: 3_000_000_000)
    # two searches of 10 levels; 1e9 algorithmic bytes a level; 1 ms and 3 ms a search of level time
    st = [_FakeStats(1.0, 10, 10_000_000, 9_360_000_000), _FakeStats(3.0, 10, 10_000_000, 9_360_000_000)]
    r = bench.roofline(st, "batched")
    alg = 64 * 10_000_000 + 9_360_000_000  # 1e10 bytes a search
    assert r["alg_bytes_per_launch"] == pytest.approx(alg / 10)
    assert r["avg_launch_ms"] == pytest.approx(0.2)  # mean 2 ms over 10 levels
    assert r["achieved"] == pytest.approx(alg / 2e-3 / 1e9)  # GB/s over the mean level time
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    assert r["traffic"] == 3_000_000_000
    assert r["traffic_GBps"] == pytest.approx(3e9 / 0.2e-3 / 1e9)
    assert r["launches_per_step"] == 10


def test_measured_traffic_follows_the_sources(tmp_path, monkeypatch):
    """A profile's bytes are reported while the hash it names is that of the current kernel
    sources, and not once a source differs or the profile is missing."""
    import hashlib

    csrc = tmp_path / "paper_1208_0274_amd" / "csrc"
    os.makedirs(csrc)
    os.makedirs(tmp_path / "profiles")
    srcs = ("level_kernels.h", "row_update.h", "device_common.h", "search.hip")
    h = hashlib.sha256()
    for f in srcs:
        shutil.copy(os.path.join(ROOT, "paper_1208_0274_amd", "csrc", f), csrc / f)
        h.update(open(csrc / f, "rb").read())
    (tmp_path / "profiles" / bench.TRAFFIC_PROFILE["batched"]).write_text(
        f"traffic_bytes_per_launch: 123456789\nsource_hash: {h.hexdigest()[:16]}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("batched") == 123456789
    assert bench.measured_traffic("long_query") is None  # no profile for it
    with open(csrc / "level_kernels.h", "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_traffic("batched") is None
