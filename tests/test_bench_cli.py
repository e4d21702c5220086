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
