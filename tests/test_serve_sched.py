"""The serving scheduler's host logic on the CPU (no GPU): tests/serve_sched_check.cpp drives
paper_1905_01348_amd/csrc/serve_sched.hpp with a simulated executor (virtual clock, workspaces
against a byte budget, injected allocation and device failures), built with g++ and the address
and undefined-behaviour sanitizers.  Checks: nearest-rank percentiles; the merge rule; a replay in
which every valid request is served once, batches never mix operations or merge classes nor pass
the pair cap or the trajectory cap, a stream never runs two batches at once, heads go oldest
first, and a second run schedules identically; V_X requests of different trajectories of one
class sharing launches (ACE requests never); a small budget, where batches wait while others run
and only a batch that cannot fit alone is refused; admission refusing arrivals with FX_ERR_BUSY
when the queue is full; cancelled requests never running; an allocation failure absorbed by one
release and retry; a device error ending the loop; an empty replay."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_serve_scheduler_with_simulated_executor(tmp_path):
    exe = str(tmp_path / "serve_sched_check")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-fno-sanitize-recover=undefined",
             "-I" + os.path.join(ROOT, "paper_1905_01348_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
             os.path.join(ROOT, "tests", "serve_sched_check.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert out.strip().splitlines()[-1].startswith("ok "), out[-2000:]
