"""The benchmark's command line on the CPU: more than one GPU is refused with a message and exit
code 2 before anything touches a GPU, and every leg and workload the contract names is offered."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_legs_and_workloads_are_offered():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for word in ("--steps", "--warmup", "--gpus", "vx", "ace", "serve", "step", "stream", "copy",
                 "24cube_16", "48cube_128", "96cube_1024x32"):
        assert word in r.stdout, word
