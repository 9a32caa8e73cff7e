"""Host-side logic of bench.py (no GPU): the one-GPU guard, and the traffic
figure that must drop to null once the kernel source no longer matches the
counters it was taken from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_source_hash_is_stable_and_tracks_the_kernel_source():
    h = bench.source_hash()
    assert h == bench.source_hash()
    assert len(h) == 12 and all(c in "0123456789abcdef" for c in h)


@pytest.mark.parametrize("matches", [True, False])
def test_traffic_is_null_once_the_source_changed(tmp_path, monkeypatch, matches):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"source_hash": bench.source_hash() if matches else "000000000000", "bytes_per_launch": 1234.0}
    (prof / "traffic_k_x_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: rec["source_hash"] if matches else "ffffffffffff")
    assert bench.load_traffic("k_x", "w") == (1234.0 if matches else None)


def test_missing_traffic_file_gives_null(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("k_none", "w") is None


def test_committed_traffic_summary_names_its_commands_and_calibration():
    path = os.path.join(ROOT, "profiles", "traffic_k_lj_force_fused_lj_bulk.json")
    rec = json.load(open(path))
    assert all(c.startswith("cd /tmp && ") and " rocprofv3 --pmc " in c and " -- python3 $R/bench.py " in c
               for c in rec["commands"])
    cal = rec["calibration"]
    # the factors scale raw counter KiB to the bytes a copy of known size
    # reads (and writes)
    size = cal["bytes_read_and_written"]
    assert cal["fetch_kib_raw"] * 1024 * cal["fetch_factor"] == pytest.approx(size, rel=1e-6)
    assert cal["write_kib_raw"] * 1024 * cal["write_factor"] == pytest.approx(size, rel=1e-6)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(
        rec["fetch_kib_per_dispatch_raw"] * 1024 * cal["fetch_factor"], rel=1e-9)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def test_cpu_baseline_record_names_the_host_and_both_thread_counts():
    from paper_1908_02038_amd import inputs
    rec = bench.cpu_baseline(inputs.lj_small(), 0.5)
    assert rec["kind"] == "oracle" and rec["unit"] == "atom-force-evals/s"
    assert rec["cores"] == rec["all_cores"]["threads"] >= 1 and rec["one_core"]["threads"] == 1
    assert rec["value"] == rec["all_cores"]["value"] > 0 and rec["one_core"]["value"] > 0
    assert rec["cpu_model"] and rec["nproc"] >= 1
    assert "cell grid" in rec["sample"]


@pytest.mark.parametrize("matches", [True, False])
def test_limiter_is_null_once_the_source_changed(tmp_path, monkeypatch, matches):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"source_hash": "abcdefabcdef", "valu_busy": 0.4, "wait_share": 0.5, "lds_wait_share": 0.02,
           "waves_per_simd": 1.5, "reading": "latency"}
    (prof / "counters_k_x_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abcdefabcdef" if matches else "ffffffffffff")
    got = bench.load_limiter("k_x", "w")
    assert (got is not None) == matches
    if matches:
        assert got["valu_busy"] == 0.4 and got["reading"] == "latency"


def test_eam_kernel_label_follows_the_tuned_tile():
    k = "k_gupta_density<float, true, true> + k_gupta_force<float, true, false>"
    assert bench.with_tile(k, "list order slot, 512-atom tiles (cached for x)") == \
        "k_gupta_density<float, true, true, 512> + k_gupta_force<float, true, false, 512>"
    assert bench.with_tile(k, "list order classes, 256-atom tiles, three blocks per CU") == \
        "k_gupta_density<float, true, true, 256> + k_gupta_force<float, true, false, 256>"
    assert bench.with_tile("k_lj_force<double, true, false, true>", "512-atom tiles") == \
        "k_lj_force<double, true, false, true>"
