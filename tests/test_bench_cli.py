"""The benchmark's command line without a GPU: more than one GPU is refused
with a message (this library measures one GPU), and every workload name in the
help text is accepted by the parser."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workload_choices():
    sys.path.insert(0, ROOT)
    import importlib
    bench = importlib.import_module("bench")
    old = sys.argv
    try:
        for w in ("cp", "batched", "nmf", "tucker", "tt", "uber", "uber400", "icews", "manybody"):
            sys.argv = ["bench.py", "--workload", w]
            assert bench.parse().workload == w
    finally:
        sys.argv = old
