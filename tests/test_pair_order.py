"""The pair enumeration of the specialised plane passes (paper_1905_01348_amd/csrc/pair_order.hpp)
on the CPU, built with g++ and the address and undefined-behaviour sanitizers: pair_of inverts
plane_of for rectangular batches and for the packed triangle of a halved apply (up to 3000
orbitals, where the float square root needs its integer correction), and the plane-forward
pass's unit order is a bijection of the batch's planes, plain and blocked (in batches of
whole blocks, each aligned run of 64 units is one block of 4 orbitals x 16 targets).  A wrong order would leave pair volumes unwritten; the GPU
parity tests would catch it only on the shapes they run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_pair_order(tmp_path):
    exe = str(tmp_path / "pair_order_check")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-fno-sanitize-recover=undefined",
             "-I" + os.path.join(ROOT, "paper_1905_01348_amd", "csrc"),
             os.path.join(ROOT, "tests", "pair_order_check.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert out.strip().splitlines()[-1].startswith("ok "), out[-2000:]
