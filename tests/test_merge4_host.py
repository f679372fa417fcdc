"""The four-way merge level on the CPU (host builds of csrc/sw_split.hpp and
csrc/sw_merge4.hpp, the code the merge kernel runs): the co-rank search
against a plain merge on every rank of small runs and on random ranks of
large ones, and a whole level -- workgroup ranges, segments, groups, split
search, rings, top-ups and final merges, thread by thread -- against a plain
sort of each group, with the rings' invariants asserted at every step.  Both
under the address and undefined-behaviour sanitizers."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name", ["split_test", "merge4_test"])
def test_four_way_merge_host(tmp_path, name):
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", name + ".cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
