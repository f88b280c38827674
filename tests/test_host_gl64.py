"""The GPU path's arithmetic compiled for the host.

gl64.h: every Goldilocks field operation against exact 128-bit arithmetic:
every shift amount of the power-of-two multiplies, edge operands (0, 1,
2^32 - 1, p - 1, p, p + 1, 2^63, 2^64 - 1, ...) and lazy operands at or
above p, which random parity inputs rarely reach.

ntt64.h: the cross-lane transform passes (forward on one wave, inverse on
one, two and four waves' lane layouts) with every lane of a wave running the
header's own code in a host thread and the lane-exchange builtins emulated,
each pass against its definition over Z_p, on random, lazy and extreme
inputs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_19871_amd", "csrc")


def test_gl64_against_128_bit_arithmetic(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "gl64_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host", "gl64_check.cpp"), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) > 1_000_000


def test_transform_passes_per_lane_layout(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "ntt_lanes_check")
    subprocess.run([cxx, "-O1", "-std=c++20", "-pthread", "-I", CSRC, os.path.join(HERE, "host", "ntt_lanes_check.cpp"),
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) >= 4 * (4 * 32 * 32 + 2 * 16 * 32 + 2 * 8 * 32)
