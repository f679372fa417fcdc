"""The oracle's pins catch plausible mistakes.

Each case compiles a copy of oracle.c with one planted mistake (a wrong sign,
a dropped byte, an unstable exchange, a wrong bucket offset, a reversed merge
comparison ...) and checks that the brute-force pins reject it.  Everything
here runs on the CPU; the shipped oracle is untouched.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1411_5283_amd import wordgen
from test_oracle import _tiny_cases, brute_force

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

MUTANTS = {
    "unstable_exchange": ("b], L) > 0;", "b], L) >= 0;"),
    "descending": ("b], L) > 0;", "b], L) < 0;"),
    "dropped_last_byte": ("chars + offsets[b], L) > 0;", "chars + offsets[b], L ? L - 1 : 0) > 0;"),
    "no_length_buckets": ("counts[word_len(offsets, i)] += 1;", "counts[0] += 1;"),
    "pass_too_short": ("for (uint32_t j = 0; j + 1 < end; ++j) {", "for (uint32_t j = 0; j + 2 < end; ++j) {"),
    "offsets_shifted": ("bucket_offsets[L] = start[L];\n    return ORC_OK;\n}\n\n/* ----",
                        "bucket_offsets[L] = start[L] + (L > 0);\n    return ORC_OK;\n}\n\n/* ----"),
    "merge_reversed": ("word_after(chars, offsets, v[head[best]], v[head[c]], (uint32_t)L)",
                       "word_after(chars, offsets, v[head[c]], v[head[best]], (uint32_t)L)"),
    "def_index_reversed": ("return a < b ? -1 : (a > b ? 1 : 0);", "return a > b ? -1 : (a < b ? 1 : 0);"),
    "def_length_ignored": ("if (la != lb)\n        return la < lb ? -1 : 1;", "if (0)\n        return 0;"),
}


def _build(tmp, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new, 1))
    so = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", path, "-o", so])
    return ctypes.CDLL(so)


def _run(lib, fname, words, chunk=None):
    wl = wordgen.from_words(words)
    chars = wl.chars if wl.chars.size else np.zeros(1, np.uint8)
    n = wl.n
    perm = np.zeros(max(n, 1), np.uint32)
    boff = np.zeros(34, np.uint32)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    args = [P(chars, ctypes.c_uint8), P(wl.offsets, ctypes.c_uint32), ctypes.c_uint32(n)]
    if chunk is not None:
        args.append(ctypes.c_uint32(chunk))
    args += [P(perm, ctypes.c_uint32), P(boff, ctypes.c_uint32)]
    getattr(lib, fname)(*args)
    return perm[:n], boff


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name):
    old, new = MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(tmp, name, old, new)
        caught = False
        for words in _tiny_cases():
            exp_perm, exp_boff = brute_force(words)
            for fname, chunk in (("oracle_bubble", None), ("oracle_def", None),
                                 ("oracle_chunked", 2), ("oracle_chunked", 3)):
                perm, boff = _run(lib, fname, words, chunk)
                if not (np.array_equal(perm, exp_perm) and np.array_equal(boff, exp_boff)):
                    caught = True
                    break
            if caught:
                break
        assert caught, "planted mistake %r passed every pin" % name
