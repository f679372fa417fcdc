"""The tokenizer's byte classes and word starts as the GPU kernels compute
them (csrc/sw_bytes.hpp: four bytes per operation, one 64-bit addition for
the starts), checked on the CPU against the reading applied byte by byte."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_token_masks_match_bytewise_reading(tmp_path):
    exe = str(tmp_path / "tok_masks_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "tok_masks_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
