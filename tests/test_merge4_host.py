"""The four-way merge pass on the CPU (host builds of csrc/sw_split.hpp and
csrc/sw_window.hpp, the code the merge kernel runs): the co-rank search
against a plain merge on every rank of small runs and on random ranks of
large ones, and the pass by bounded windows -- bound, counts by the two probe
rounds, the merges of every step, the window loads -- walked from random
start ranks over groups of many shapes against a plain sort.  Both under the
address and undefined-behaviour sanitizers."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name", ["split_test", "window_test"])
def test_four_way_merge_host(tmp_path, name):
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", name + ".cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
