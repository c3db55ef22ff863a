"""The blocked face-plane layout of the sweep kernels, checked on the host: a small C++
program (tests/face_layout_check.cpp) includes the layout from the library's internal
header, gives every vertex of a slot its own position, simulates the writes of the
ghost fill and of the tiles, and checks that every tile's incoming face (interior,
halo row and column, as the kernels address them) reads the vertices expected."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_face_layout(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "face_layout_check")
    subprocess.run([hipcc, "-std=c++17", "-O1", os.path.join(HERE, "face_layout_check.cpp"), "-o", exe], check=True,
                   capture_output=True)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0 and run.stdout.strip().endswith("OK"), run.stdout
