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
from test_oracle import _tiny_cases, brute_force, chunks_brute_force

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


# Planted mistakes in oracle_length_counts: an index off by one, a word
# skipped at either end of the loop, the byte at the start counted instead of
# the length, the error check dropped for long words (they would then be
# counted past the last list, so the mutant clamps them the way an earlier
# version did).
COUNT_MUTANTS = {
    "index_minus_one": ("counts[offsets[i + 1] - offsets[i]] += 1;",
                        "counts[offsets[i + 1] - offsets[i] - (offsets[i + 1] > offsets[i])] += 1;"),
    "index_plus_one": ("counts[offsets[i + 1] - offsets[i]] += 1;",
                       "counts[offsets[i + 1] - offsets[i] + (offsets[i + 1] - offsets[i] < 32)] += 1;"),
    "first_word_skipped": ("    for (uint32_t i = 0; i < n; ++i)\n        counts[offsets[i + 1]",
                           "    for (uint32_t i = 1; i < n; ++i)\n        counts[offsets[i + 1]"),
    "last_word_skipped": ("    for (uint32_t i = 0; i < n; ++i)\n        counts[offsets[i + 1]",
                          "    for (uint32_t i = 0; i + 1 < n; ++i)\n        counts[offsets[i + 1]"),
    "offset_not_length": ("counts[offsets[i + 1] - offsets[i]] += 1;",
                          "counts[offsets[i + 1] % 33] += 1;"),
    "long_words_clamped": ("    const int rc = check_words(offsets, n);\n    if (rc != ORC_OK)\n        return rc;\n"
                           "    for (int L = 0; L < ORC_NBUCKET; ++L)\n        counts[L] = 0;\n"
                           "    for (uint32_t i = 0; i < n; ++i)\n        counts[offsets[i + 1] - offsets[i]] += 1;",
                           "    for (int L = 0; L < ORC_NBUCKET; ++L)\n        counts[L] = 0;\n"
                           "    for (uint32_t i = 0; i < n; ++i)\n        counts[offsets[i + 1] - offsets[i] > 32 ? 32 : "
                           "offsets[i + 1] - offsets[i]] += 1;"),
}


def _length_counts(lib, offsets):
    offsets = np.ascontiguousarray(offsets, np.uint32)
    out = np.zeros(33, np.uint64)
    lib.oracle_length_counts.restype = ctypes.c_int
    rc = lib.oracle_length_counts(offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                  ctypes.c_uint32(offsets.shape[0] - 1),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return rc, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(COUNT_MUTANTS))
def test_length_count_pins_reject_mutant(name):
    old, new = COUNT_MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(tmp, name, old, new)
        caught = False
        # the pins of test_oracle.py: bincount on generated text, closed forms,
        # the brute-force bucket sizes, the error code for a long word
        wl = wordgen.config(1, 0.2)
        rc, got = _length_counts(lib, wl.offsets)
        caught |= rc != 0 or not np.array_equal(got, np.bincount(np.diff(wl.offsets.astype(np.int64)),
                                                                 minlength=33))
        lens = np.arange(33)
        rc, got = _length_counts(lib, np.concatenate([[0], np.cumsum(lens)]))
        caught |= rc != 0 or not np.array_equal(got, np.ones(33, np.uint64))
        for words in list(_tiny_cases())[:50]:
            w = wordgen.from_words(words)
            _, boff = brute_force(words)
            rc, got = _length_counts(lib, w.offsets)
            caught |= rc != 0 or not np.array_equal(got, np.diff(boff.astype(np.int64))[:33])
        rc, _ = _length_counts(lib, np.array([0, 33], np.uint32))
        caught |= rc != -2
        assert caught, "planted mistake %r passed every pin" % name


# Planted mistakes in the chunk step alone (oracle_chunks): chunk boundaries
# shifted, the last chunk cut short, a chunk one word too long.
CHUNK_MUTANTS = {
    "chunk_stride_plus_one": ("for (uint32_t lo = 0; lo < counts[L]; lo += chunk) {",
                              "for (uint32_t lo = 0; lo < counts[L]; lo += chunk + 1) {"),
    "chunk_starts_at_one": ("for (uint32_t lo = 0; lo < counts[L]; lo += chunk) {",
                            "for (uint32_t lo = counts[L] > chunk; lo < counts[L]; lo += chunk) {"),
    "last_chunk_short": ("uint32_t len = (counts[L] - lo < chunk) ? counts[L] - lo : chunk;",
                         "uint32_t len = (counts[L] - lo < chunk) ? counts[L] - lo - (counts[L] - lo > 1) : chunk;"),
    "chunk_one_too_long": ("uint32_t len = (counts[L] - lo < chunk) ? counts[L] - lo : chunk;",
                           "uint32_t len = (counts[L] - lo <= chunk) ? counts[L] - lo : chunk + 1;"),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(CHUNK_MUTANTS))
def test_chunk_step_pins_reject_mutant(name):
    old, new = CHUNK_MUTANTS[name]
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(tmp, name, old, new)
        caught = False
        for words in _tiny_cases():
            for c in (1, 2, 3):
                exp_perm, exp_boff = chunks_brute_force(words, c)
                perm, boff = _run(lib, "oracle_chunks", words, c)
                if not (np.array_equal(perm, exp_perm) and np.array_equal(boff, exp_boff)):
                    caught = True
                    break
            if caught:
                break
        assert caught, "planted mistake %r passed every pin" % name
