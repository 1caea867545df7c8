"""Host-side logic of bench.py (CPU, no GPU calls): the one-GPU guard and the
rule for reporting counter-measured traffic."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_reason():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_reported_only_for_the_recorded_kernel_and_launch(tmp_path):
    bench = _bench_module()
    src = os.path.join(ROOT, "paper_1502_07873_amd", "csrc", "stencil.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    rec = {"kernel_source_sha256": sha, "solves_per_launch": 24, "variant": 9,
           "wave_cache_bytes": 192 << 20, "traffic_bytes_per_launch": 1.5e8}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    bench.TRAFFIC_RECORD = str(path)
    assert bench._measured_traffic(24, 192 << 20, 9) == 1.5e8
    assert bench._measured_traffic(23, 192 << 20, 9) is None     # other launch size
    assert bench._measured_traffic(24, 0, 9) is None             # unsplit waves
    assert bench._measured_traffic(24, 192 << 20, 10) is None    # other tile shape
    rec["kernel_source_sha256"] = "0" * 64                        # kernel changed since
    path.write_text(json.dumps(rec))
    assert bench._measured_traffic(24, 192 << 20, 9) is None
    bench.TRAFFIC_RECORD = str(tmp_path / "missing.json")
    assert bench._measured_traffic(24, 192 << 20, 9) is None


def test_committed_traffic_record_matches_the_kernel_source():
    # the record under profiles/ must describe the stencil source as it is
    rec = json.load(open(os.path.join(ROOT, "profiles", "stencil_layered_c2_traffic.json")))
    src = os.path.join(ROOT, "paper_1502_07873_amd", "csrc", "stencil.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec["kernel_source_sha256"] != sha:
        pytest.xfail("stencil.hip changed since the counters were taken: bench reports "
                     "traffic null until they are taken again")
    assert rec["traffic_bytes_per_launch"] >= rec["kernel_floor_bytes_per_launch_16B_per_update"]
