"""bench.py's command line without a GPU: more than one GPU is refused with a
message before any device work; the walk-source hash used to match stored
traffic counters is printable."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_walk_hash_prints():
    r = _run("--print-walk-hash")
    assert r.returncode == 0
    h = r.stdout.strip()
    assert len(h) == 16 and int(h, 16) >= 0


def test_traffic_profile_used_only_for_matching_sources(tmp_path, monkeypatch):
    # The stored DRAM-traffic record is reported only while the walk sources
    # hash as they did when the counters were taken; else it is null.
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    h = bench.walk_source_hash()
    prof = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic() is None                      # no profile
    prof.write_text('text\nTRAFFIC_JSON {"walk_source_hash": "%s", "l2_to_memory_bytes_per_launch": 123.5, '
                    '"launch_ms": 2.0}\n' % h)
    assert bench.measured_traffic()["l2_to_memory_bytes_per_launch"] == 123.5
    prof.write_text('TRAFFIC_JSON {"walk_source_hash": "0000000000000000", "l2_to_memory_bytes_per_launch": 1}\n')
    assert bench.measured_traffic() is None                      # taken on other kernel sources
    prof.write_text('TRAFFIC_JSON {not json}\n')
    assert bench.measured_traffic() is None


def test_probe_cases_stay_inside_their_buffer():
    # every probe window starts below its region and the buffer holds
    # region + window bytes, so no load leaves the allocation
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    need = max(c[3] + c[4] for c in bench.PROBE_CASES)
    for name, kind, width, region, window, stride in bench.PROBE_CASES:
        if kind:
            continue
        assert window >= 256 * width * 4, name          # one round of a workgroup fits the window
        assert region + window <= need and region < 2 ** 32 and window < 2 ** 31, name
