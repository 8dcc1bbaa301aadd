"""Host-side parts of the benchmark: the one-GPU guard and the lookup of the
committed HBM-traffic figure, which is void once the kernel sources change."""
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(path, sha, nbytes):
    path.write_text("# counters\n\n"
                    f"- `kernel_sources_sha256: {sha}`\n"
                    f"- `hbm_bytes_per_launch: {nbytes}`\n")


def test_traffic_read_only_for_unchanged_kernel(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))
    _summary(f, bench.kernel_sources_sha256(), 123456.5)
    assert bench.force_traffic("plummer_n16384") == 123456.5
    assert bench.force_traffic("plummer_n1024") is None
    _summary(f, "0" * 64, 123456.5)
    assert bench.force_traffic("plummer_n16384") is None


def test_traffic_missing_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.md"))
    assert bench.force_traffic("plummer_n16384") is None


def test_cpu_baseline_fields():
    """The oracle leg on a tiny workload: both rates positive, the thread
    count and the host description reported."""
    w = {"n": 64, "seed": 1, "eps": 1e-4, "eta": 0.01, "dt_max": 0.125, "dt_min": 2.0 ** -22, "t_end": 0.125}
    cb = bench.cpu_baseline(w, 0.3)
    assert cb["kind"] == "oracle" and cb["unit"] == "pair-interactions/s"
    assert cb["value"] > 0 and cb["single_thread"]["value"] > 0
    assert cb["cores"] >= 1 and cb["usable_cpus"] >= 1
    assert "block steps" in cb["sample"] and "block steps" in cb["single_thread"]["sample"]
