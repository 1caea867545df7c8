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
    sha = bench._sources_sha(*bench.LAYERED_SOURCES)
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
    # the four-step kernel's record is keyed to its own sources
    rec = {"kernel_source_sha256": bench._sources_sha(*bench.BLOCKED_SOURCES),
           "solves_per_launch": 3840, "variant": 23, "wave_cache_bytes": 192 << 20,
           "traffic_bytes_per_launch": 3.9e10}
    path.write_text(json.dumps(rec))
    bench.TRAFFIC_RECORD = str(path)
    assert bench._measured_traffic(3840, 192 << 20, 23) == 3.9e10
    rec["kernel_source_sha256"] = sha                             # the tiled kernels' hash
    path.write_text(json.dumps(rec))
    assert bench._measured_traffic(3840, 192 << 20, 23) is None


@pytest.mark.parametrize("record,tiled", [("stencil_layered_c2_traffic.json", "LAYERED_SOURCES"),
                                          ("stencil_nodal_c5_traffic.json", "NODAL_SOURCES"),
                                          ("stencil_resident_model_problem.json",
                                           "RESIDENT_SOURCES")])
def test_committed_counter_records_match_the_kernel_sources(record, tiled):
    # each record under profiles/ names the sources of its variant's kernel
    # (the ones bench.py hashes for that variant) and must describe them as
    # they are (else the bench reports its traffic as null)
    bench = _bench_module()
    rec = json.load(open(os.path.join(ROOT, "profiles", record)))
    sources = bench._kernel_sources(rec["variant"], getattr(bench, tiled))
    assert tuple(rec["sources"]) == sources
    if rec["kernel_source_sha256"] != bench._sources_sha(*sources):
        pytest.xfail(f"{sources} changed since the counters of {record} were taken: bench "
                     "reports their figures as null until they are taken again")
    traffic = rec.get("traffic_bytes_per_launch", rec.get("traffic_bytes_per_update"))
    assert traffic > 0
    assert traffic >= rec.get("kernel_floor_bytes_per_launch", 0)


def test_variant_steps_and_kernel_sources():
    # the bench labels a launch by its variant: steps per launch for the
    # solves-per-launch and floor arithmetic, and the kernel's own source
    # files for the counter-record hash
    bench = _bench_module()
    assert [bench._steps_per_launch(v) for v in (0, 6, 8, 9, 14, 15, 16, 18, 19, 20)] == \
        [1, 1, 1, 2, 2, 3, 3, 1, 2, 2]
    assert [bench._steps_per_launch(v) for v in (23, 24, 25)] == [4, 4, 4]
    for v in (23, 24, 25):
        assert bench._kernel_sources(v, bench.LAYERED_SOURCES) == bench.BLOCKED_SOURCES
        assert bench._kernel_sources(v, bench.NODAL_SOURCES) == bench.BLOCKED_SOURCES
    assert bench._kernel_sources(9, bench.LAYERED_SOURCES) == bench.LAYERED_SOURCES
    assert bench._kernel_sources(20, bench.NODAL_SOURCES) == bench.NODAL_SOURCES
    assert bench.BLOCKED_FLOOR_B == 8.0
