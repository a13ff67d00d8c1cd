"""The brick geometry of the pair passes on the CPU (paper_2103_08932_amd/csrc/bricks.hpp compiled
with g++ against the mock HIP header, with AddressSanitizer and UndefinedBehaviorSanitizer): on random
2D and 3D cell grids with empty cells, for brick lengths 1-5 and 8 and the column and tiled brick
orders, every brick is visited once, its runs hold exactly the particles of the cells within one cell
of it (found by walking the cells), its first run sits at offset zero, the run records that setup
stores read back to the same runs, and the XCD remap launches every brick once
(tests/bricks_host/bricks_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_brick_geometry_and_run_records(tmp_path):
    exe = str(tmp_path / "bricks_check")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           f"-I{os.path.join(ROOT, 'tests', 'server_mock')}",
           f"-I{os.path.join(ROOT, 'paper_2103_08932_amd', 'csrc')}",
           os.path.join(ROOT, "tests", "bricks_host", "bricks_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "bricks ok" in r.stdout
