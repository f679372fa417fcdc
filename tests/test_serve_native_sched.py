"""The native serving scheduler's rules (csrc/sw_sched.hpp), on the CPU: a
C++ test with a stand-in executor and a simulated clock checks FIFO
admission under the HBM budget (the head is never overtaken), batch limits
and order, overlap of the two slots, failure isolation and the intake
checks."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_native_scheduler_rules(tmp_path):
    exe = str(tmp_path / "sched_test")
    # host-only code: built with g++ under the address and undefined-behaviour sanitizers
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I",
                           os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "sched_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
