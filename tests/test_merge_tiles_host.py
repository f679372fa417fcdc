"""The two-way merge levels' tile geometry (csrc/sw_tiles.hpp: merge_tile,
tile_io, the placement bookkeeping of a workgroup's range, the K-ary segment
search), the code the merge kernel runs, built for the host with g++ under
the address and undefined-behaviour sanitizers: every tile of random
segments at every level reads inside its pair of runs without clamping and
merges exactly the outputs it owns (against a plain merge), the ranges give
every tile its record and its successor's split, and the search finds every
tile's segment."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_merge_tile_geometry(tmp_path):
    exe = str(tmp_path / "tiles_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "tiles_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
