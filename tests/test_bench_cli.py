"""bench.py contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as fh:
        fh.write('"Kernel_Name","Counter_Name","Counter_Value"\n')
        for k, v in rows:
            fh.write(f'"{k}","{counter}",{v}\n')


def test_summarize_pmc_calibrates_against_the_copy(tmp_path, monkeypatch):
    """HBM bytes per dispatch = median raw count x (256 MiB / the copy's count), per counter,
    written with the kernel-source hash; a kernel missing from either run is skipped."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "kernel_src_sha", lambda: "abc123")
    sweep = bench.PMC_KERNELS["swe_sweep_p4_256x256"]
    copy = "__amd_rocclr_copyBuffer"
    # FETCH_SIZE reads half the copy's bytes (factor 2), WRITE_SIZE all of them (factor 1)
    _write_counters(tmp_path / "f", "FETCH_SIZE",
                    [(copy, 131072.0), (sweep + "(args)", 100.0), (sweep + "(args)", 300.0), (sweep + "(args)", 200.0)])
    _write_counters(tmp_path / "w", "WRITE_SIZE", [(copy, 262144.0), (sweep + "(args)", 50.0)])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"))
    d = json.load(open(tmp_path / "profiles" / "swe_sweep_p4_256x256_pmc.json"))
    assert d["kernel_src_sha"] == "abc123"
    assert d["dispatches"] == [3, 1]
    assert d["copy_calibration"]["fetch_factor"] == 2.0 and d["copy_calibration"]["write_factor"] == 1.0
    assert d["hbm_bytes_per_dispatch"] == (200.0 * 2.0 + 50.0 * 1.0) * 1024.0
    assert not os.path.exists(tmp_path / "profiles" / "swe_step_p4_256x256_pmc.json")


def test_traffic_is_reported_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    with open(tmp_path / "profiles" / "t_pmc.json", "w") as fh:
        json.dump({"kernel_src_sha": "abc123", "hbm_bytes_per_dispatch": 123.0}, fh)
    monkeypatch.setattr(bench, "kernel_src_sha", lambda: "abc123")
    assert bench.traffic_from_profiles("t", 1) == 123.0
    monkeypatch.setattr(bench, "kernel_src_sha", lambda: "other")
    assert bench.traffic_from_profiles("t", 1) is None
    assert bench.traffic_from_profiles("missing", 1) is None
