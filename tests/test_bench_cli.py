"""bench.py's command line on the host: one GPU only, and every workload name
accepted by the parser."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("poisson1024", "wilson256", "wilson512", "varcoef_batch", "graph1m",
              "laplace_bilinear", "gauge256"):
        assert w in r.stdout
