"""The sorted-text kernel's dword writer (csrc/sw_bytes.hpp: a word's text
from its key lanes, whole dwords inside the word, bytes and halfwords at its
edges), checked on the CPU against the text written byte by byte: every
length, start offset and separator, lanes with garbage past the word, and
runs of words written back to back in random order."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_word_text_dwords_match_bytewise_text(tmp_path):
    exe = str(tmp_path / "word_text_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1411_5283_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "word_text_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
