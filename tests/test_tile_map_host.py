"""The block -> tile maps of the hop kernels (hop.hpp), checked on the CPU: a small host
program compiled from tests/tile_map_check.hip against the library's own header walks every
block of the grid that tile_map_blocks sizes and checks that each (tile, right-hand-side
group) pair is covered exactly once, for every map, run of time slices, block size and group
count on ragged and regular lattices.  Nothing runs on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_tile_maps_cover_every_tile_once(tmp_path):
    exe = str(tmp_path / "tile_map_check")
    src = os.path.join(ROOT, "tests", "tile_map_check.hip")
    inc = [os.path.join(ROOT, "paper_2502_03249_amd", "csrc"), os.path.join(ROOT, "include")]
    cmd = [HIPCC, "-x", "hip", "-std=c++17", "-O1", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops"] + [f"-I{d}" for d in inc] + [src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "bad 0" in r.stdout
