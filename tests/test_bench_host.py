"""Host-side checks of the benchmark script: the one-GPU contract and the lookup of the
committed HBM-traffic records (valid only while the kernel source is unchanged)."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_peak_is_the_alu_roof():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, 2.5 lane-instructions per minimal Joseph update
    assert abs(bench.PEAK_UPDATES - 256 * 4 * 16 * 2.4e9 / 2.5) <= 1e-6 * bench.PEAK_UPDATES
    r = bench.alu_roofline("fp_kernel", 1e9, 100.0)
    assert abs(r["frac"] - 1e13 / bench.PEAK_UPDATES) < 1e-12
    assert abs(r["valu_frac_at_4_5"] - 1e13 * 4.5 / (256 * 4 * 16 * 2.4e9)) < 1e-12


def _record(h, nbytes):
    return "traffic-json: " + json.dumps({
        "workload": "single-roi-1024", "kernel": "bp_kernel", "kernel_source_sha256": h,
        "bytes_per_launch": nbytes})


def test_traffic_record_needs_the_current_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    h = bench.kernel_source_hash()
    (prof / "bp.md").write_text("# summary\n\n" + _record("0" * 16, 111) + "\n" +
                                _record(h, 2315898) + "\n")
    assert bench.profiled_traffic("single-roi-1024", "bp_kernel") == 2315898
    assert bench.profiled_traffic("single-roi-1024", "fp_kernel") is None
    # any edit of the kernel source voids the record
    src.write_text("// kernel source, changed\n")
    assert bench.profiled_traffic("single-roi-1024", "bp_kernel") is None


def _committed_records():
    recs = []
    prof = os.path.join(ROOT, "profiles")
    for fn in sorted(os.listdir(prof)):
        if fn.endswith(".md"):
            with open(os.path.join(prof, fn)) as f:
                recs += [(fn, json.loads(line[len("traffic-json: "):]))
                         for line in f if line.startswith("traffic-json: ")]
    return recs


def test_committed_traffic_records_are_consistent():
    recs = _committed_records()
    assert recs
    # one set, all taken on one kernel source
    assert len({r["kernel_source_sha256"] for _, r in recs}) == 1
    keys = {(r["workload"], r["kernel"]) for _, r in recs}
    assert len(keys) == len(recs)
    # the pairs the benchmark looks up
    for key in [("tiles256-n4096-a512", "bp_kernel"), ("batch64-n2048-a256", "bp_kernel"),
                ("single-roi-1024", "bp_kernel"), ("single-roi-1024", "fp_kernel"),
                ("batch64-n2048-a256-alg2", "bp_kernel (two-channel)")]:
        assert key in keys, key
    for fn, r in recs:
        # bytes = FETCH_SIZE x scale + WRITE_SIZE x scale, the counters printed to 0.1 KiB
        est = 1024.0 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])
        tol = 0.05 * 1024.0 * (r["fetch_scale"] + r["write_scale"]) + 1.0
        assert abs(r["bytes_per_launch"] - est) <= tol, (fn, r["kernel"])
        # the copy calibration: on a 256 MiB copy FETCH_SIZE counts half of the bytes read,
        # WRITE_SIZE all of those written
        assert abs(r["fetch_scale"] - 2.0) < 0.01 and abs(r["write_scale"] - 1.0) < 0.01
        # a unit slip (KiB taken for bytes, a scale left out) would put the bytes far below
        # the kernel's algorithmic bytes
        assert r["bytes_per_launch"] > 0.5 * r["algorithmic_bytes_per_launch"], (fn, r["kernel"])
