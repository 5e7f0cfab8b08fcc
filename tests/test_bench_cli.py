"""bench.py's command line on the CPU: one GPU only, and the workload list."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    env = dict(os.environ, WORLD_SIZE="4")
    r = _run(env=env)
    assert r.returncode == 2


def test_workloads_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("paper224", "mixed", "proposal", "crossover"):
        assert w in r.stdout
