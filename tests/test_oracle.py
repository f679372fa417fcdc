"""Pins of the CPU oracle against what the paper and the mathematics fix.

* brute force: over all n! orderings of tiny inputs exactly one is strictly
  increasing under (length, bytes, index); every oracle must return it;
* Python's ``sorted`` (stable by definition) and qsort under the total order;
* invariants at any size, closed forms, the error codes;
* the paper's printed numbers: the chunk-size example (section 5) and the
  derived columns of Tables 1 and 3.
"""
import itertools
import os

import numpy as np
import pytest

from checks import check_invariants
from paper_1411_5283_amd import report, wordgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_force(words):
    n = len(words)
    keys = [(len(w), w, i) for i, w in enumerate(words)]
    hits = [p for p in itertools.permutations(range(n))
            if all(keys[p[k]] < keys[p[k + 1]] for k in range(n - 1))]
    assert len(hits) == 1
    boff = [sum(1 for w in words if len(w) < L) for L in range(34)]
    return np.asarray(hits[0], np.uint32), np.asarray(boff, np.uint32)


TINY = [b"", b"a", b"b", b"aa", b"ab", b"ba", b"bb", b"aab", b"bba", b"abb"]


def _tiny_cases():
    # exhaustive over 3-word sequences of a 6-word set, plus seeded samples up to n=7
    for seq in itertools.product(TINY[:6], repeat=3):
        yield list(seq)
    rng = np.random.default_rng(5283)
    for n in range(1, 8):
        for _ in range(60 if n < 7 else 12):
            yield [TINY[k] for k in rng.integers(0, len(TINY), n)]
    # heavy duplicates and reversed orders
    yield [b"b", b"b", b"a", b"a", b"b", b"a"]
    yield [b"bb", b"ba", b"ab", b"aa", b"b", b"a", b""]


def test_brute_force_pins_every_oracle(oracle_mod):
    for words in _tiny_cases():
        wl = wordgen.from_words(words)
        exp_perm, exp_boff = brute_force(words)
        for fn in (oracle_mod.oracle_bubble, oracle_mod.oracle_def):
            perm, boff = fn(wl.chars, wl.offsets)
            assert np.array_equal(perm, exp_perm), (fn.__name__, words)
            assert np.array_equal(boff, exp_boff), (fn.__name__, words)
        for c in range(1, len(words) + 2):
            perm, boff = oracle_mod.oracle_chunked(wl.chars, wl.offsets, c)
            assert np.array_equal(perm, exp_perm), ("chunked", c, words)
            assert np.array_equal(boff, exp_boff)
        perm, boff = oracle_mod.oracle_sorted(words)
        assert np.array_equal(perm, exp_perm) and np.array_equal(boff, exp_boff)


def test_unsigned_byte_order(oracle_mod):
    # bytes compare as unsigned: 0xff sorts after 0x01 and 'z'; byte 0 sorts first
    words = [b"\xff", b"\x01", b"z", b"\x00", b"\x80\x00", b"\x7f\xff", b"\x00\x00"]
    wl = wordgen.from_words(words)
    exp, _ = brute_force(words)
    for fn in (oracle_mod.oracle_bubble, oracle_mod.oracle_def):
        perm, _ = fn(wl.chars, wl.offsets)
        assert np.array_equal(perm, exp)
    assert list(exp) == [3, 1, 2, 0, 6, 5, 4]


@pytest.mark.parametrize("scale_cfg", [(1, 1.0), (2, 0.3)])
def test_oracles_agree_on_generated_text(oracle_mod, scale_cfg):
    cfg, scale = scale_cfg
    wl = wordgen.config(cfg, scale)
    p1, b1 = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    p2, b2 = oracle_mod.oracle_def(wl.chars, wl.offsets)
    assert np.array_equal(p1, p2) and np.array_equal(b1, b2)
    check_invariants(wl.chars, wl.offsets, p1, b1)
    if cfg == 1:
        p3, b3 = oracle_mod.oracle_sorted(wl.words())
        assert np.array_equal(p1, p3) and np.array_equal(b1, b3)
        p4, b4 = oracle_mod.oracle_chunked(wl.chars, wl.offsets, 1024)
        assert np.array_equal(p1, p4) and np.array_equal(b1, b4)


def test_closed_forms(oracle_mod):
    # all words equal -> identity
    wl = wordgen.from_words([b"same"] * 50)
    perm, boff = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    assert np.array_equal(perm, np.arange(50)) and boff[4] == 0 and boff[5] == 50
    # input already in key order -> identity
    words = [b"", b"a", b"a", b"b", b"ab", b"ba", b"abc", b"abd", b"zzzz"]
    wl = wordgen.from_words(words)
    perm, _ = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    assert np.array_equal(perm, np.arange(len(words)))
    # distinct equal-length words in reverse order -> reversed identity
    words = [bytes([100 - k, 65 + (k % 3)]) for k in range(40)]
    wl = wordgen.from_words(words)
    perm, _ = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    assert np.array_equal(perm, np.arange(39, -1, -1))
    # all lengths distinct -> stable argsort of the lengths
    rng = np.random.default_rng(1)
    lens = rng.permutation(33)
    words = [bytes(rng.integers(0, 256, L, dtype=np.uint8)) for L in lens]
    wl = wordgen.from_words(words)
    perm, boff = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    assert np.array_equal(perm, np.argsort(lens, kind="stable"))
    assert np.array_equal(boff, np.arange(34))


def test_empty_and_zero_length(oracle_mod):
    perm, boff = oracle_mod.oracle_bubble(np.zeros(0, np.uint8), np.zeros(1, np.uint32))
    assert perm.shape[0] == 0 and np.all(boff == 0)
    wl = wordgen.from_words([b"", b"", b""])
    perm, boff = oracle_mod.oracle_bubble(wl.chars, wl.offsets)
    assert list(perm) == [0, 1, 2] and boff[0] == 0 and boff[1] == 3 and boff[33] == 3


def test_error_codes(oracle_mod):
    wl = wordgen.from_words([b"a" * 32, b"b"])
    assert oracle_mod.oracle_status(wl.chars, wl.offsets) == oracle_mod.OK
    wl = wordgen.from_words([b"a" * 33, b"b"])
    for fn in ("oracle_bubble", "oracle_def"):
        assert oracle_mod.oracle_status(wl.chars, wl.offsets, fn) == oracle_mod.WORD_TOO_LONG
    bad = np.array([0, 5, 3, 40], np.uint32)           # decreases, and a 37-byte word
    chars = np.zeros(40, np.uint8)
    for fn in ("oracle_bubble", "oracle_def"):
        assert oracle_mod.oracle_status(chars, bad, fn) == oracle_mod.INVALID_ARG


def test_nonzero_first_offset(oracle_mod):
    # offsets[0] need not be 0: words are read where the offsets point
    base = wordgen.from_words([b"cab", b"ab", b"ca", b"a"])
    chars = np.concatenate([np.frombuffer(b"XXXX", np.uint8), base.chars])
    offs = base.offsets + 4
    perm, boff = oracle_mod.oracle_bubble(chars, offs)
    assert list(perm) == [3, 1, 2, 0]


def test_rank_matches_sort(oracle_mod):
    wl = wordgen.config(1, 0.05)
    perm, _ = oracle_mod.oracle_def(wl.chars, wl.offsets)
    for i in [0, 1, 17, wl.n // 2, wl.n - 1]:
        assert perm[oracle_mod.oracle_rank(wl.chars, wl.offsets, i)] == i


def test_batch_oracle_is_per_document(oracle_mod):
    docs = [wordgen.config(1, 0.01), wordgen.from_words([b"b", b"a"]),
            wordgen.from_words([]), wordgen.config(2, 0.004)]
    wl = wordgen.concat_docs(docs)
    perm, boff = oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets)
    for d, doc in enumerate(docs):
        lo, hi = int(wl.doc_offsets[d]), int(wl.doc_offsets[d + 1])
        p, b = oracle_mod.oracle_sorted(doc.words())
        assert np.array_equal(perm[lo:hi], p) and np.array_equal(boff[d], b)


# ----------------------------------------------------------------- paper's numbers
def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_paper_chunk_example(oracle_mod):
    for size, p, chunk in _rows("paper_chunk_example.txt"):
        assert oracle_mod.paper_chunk_size(int(size), int(p)) == int(chunk)


def test_paper_table1_average():
    rows = _rows("paper_table1.txt")
    runs = [r for r in rows if r[0] != "ave"]
    ave = [r for r in rows if r[0] == "ave"][0]
    for col in (1, 2):
        m = report.mean(r[col] for r in runs)
        assert abs(m - float(ave[col])) < 1e-3      # printed to three decimals


def test_paper_table3_derived_columns():
    rows = _rows("paper_table3.txt")
    t1 = {1: float(rows[0][1]), 2: float(rows[0][2])}
    for r in rows:
        p = int(r[0])
        for d, (tc, sc, ec) in {1: (1, 3, 5), 2: (2, 4, 6)}.items():
            tp = float(r[tc])
            assert abs(report.speedup(t1[d], tp) - float(r[sc])) < 1e-3
            assert abs(report.efficiency(t1[d], tp, p) - float(r[ec])) < 1e-3


def test_invariant_checker_rejects_wrong_orders(oracle_mod):
    wl = wordgen.config(1, 0.05)
    perm, boff = oracle_mod.oracle_def(wl.chars, wl.offsets)
    check_invariants(wl.chars, wl.offsets, perm, boff)
    lens = np.diff(wl.offsets.astype(np.int64))
    # swap two neighbours of equal length (a byte- or index-order violation)
    k = next(k for k in range(len(perm) - 1) if lens[perm[k]] == lens[perm[k + 1]])
    bad = perm.copy()
    bad[k], bad[k + 1] = bad[k + 1], bad[k]
    with pytest.raises(AssertionError):
        check_invariants(wl.chars, wl.offsets, bad, boff)
    bad = perm.copy()
    bad[-1] = bad[0]                                   # not a permutation
    with pytest.raises(AssertionError):
        check_invariants(wl.chars, wl.offsets, bad, boff)
    badb = boff.copy()
    badb[5] += 1                                       # bucket offset off by one
    with pytest.raises(AssertionError):
        check_invariants(wl.chars, wl.offsets, perm, badb)


# ---------------------------------------------------------------- length counts
# oracle_length_counts gives the sizes of the phase-2 lists (Abstract: one
# sub-array per character count, sized by how many words have that count).
# Pinned against numpy's bincount (a library routine), closed forms, the
# bucket offsets that the brute force fixes, and its error codes.

@pytest.mark.parametrize("cfg,scale", [(1, 1.0), (2, 0.5), (4, 0.002)])
def test_length_counts_equal_bincount(oracle_mod, cfg, scale):
    wl = wordgen.config(cfg, scale)
    lens = np.diff(wl.offsets.astype(np.int64))
    exp = np.bincount(lens, minlength=33)
    got = oracle_mod.oracle_length_counts(wl.offsets)
    assert got.shape == (33,) and np.array_equal(got, exp)
    assert int(got.sum()) == wl.n


def test_length_counts_closed_forms(oracle_mod):
    # n empty words: everything in list 0
    got = oracle_mod.oracle_length_counts(np.zeros(1001, np.uint32))
    assert got[0] == 1000 and not got[1:].any()
    # every length 0..32 once, in either order: all ones
    for lens in (np.arange(33), np.arange(33)[::-1]):
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint32)
        assert np.array_equal(oracle_mod.oracle_length_counts(offs), np.ones(33, np.uint64))
    # a non-zero first offset changes nothing
    offs = np.array([7, 7, 9, 9, 41, 44], np.uint32)      # lengths 0, 2, 0, 32, 3
    exp = np.zeros(33, np.uint64)
    exp[[0, 2, 32, 3]] = [2, 1, 1, 1]
    assert np.array_equal(oracle_mod.oracle_length_counts(offs), exp)
    # no words at all
    assert not oracle_mod.oracle_length_counts(np.array([5], np.uint32)).any()


def test_length_counts_are_the_brute_force_bucket_sizes(oracle_mod):
    for words in _tiny_cases():
        wl = wordgen.from_words(words)
        _, boff = brute_force(words)
        got = oracle_mod.oracle_length_counts(wl.offsets)
        assert np.array_equal(got, np.diff(boff.astype(np.int64))[:33]), words


def test_length_counts_error_codes(oracle_mod):
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.oracle_length_counts(np.array([0, 33], np.uint32))
    assert e.value.code == oracle_mod.WORD_TOO_LONG
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.oracle_length_counts(np.array([0, 40, 5], np.uint32))   # decreases and too long
    assert e.value.code == oracle_mod.INVALID_ARG
    assert oracle_mod.oracle_length_counts(np.array([0, 32], np.uint32))[32] == 1


def chunks_brute_force(words, chunk):
    """The chunk step by brute force: each length list (input order) cut into
    chunks of `chunk` from its start, each chunk ordered by the one strictly
    increasing permutation of its (bytes, index) keys."""
    out = []
    for L in range(33):
        lst = [i for i, w in enumerate(words) if len(w) == L]
        for lo in range(0, len(lst), chunk):
            part = lst[lo:lo + chunk]
            local, _ = brute_force([words[i] for i in part])
            out += [part[k] for k in local]
    boff = [sum(1 for w in words if len(w) < L) for L in range(34)]
    return np.asarray(out, np.uint32), np.asarray(boff, np.uint32)


def test_chunk_step_pins(oracle_mod):
    # brute force per chunk on the tiny cases, every chunk size that matters
    for words in list(_tiny_cases())[::3]:
        wl = wordgen.from_words(words)
        for c in range(1, len(words) + 2):
            exp_perm, exp_boff = chunks_brute_force(words, c)
            perm, boff = oracle_mod.oracle_chunks(wl.chars, wl.offsets, c)
            assert np.array_equal(perm, exp_perm), (c, words)
            assert np.array_equal(boff, exp_boff)
    wl = wordgen.config(1, 0.1)
    lens = np.diff(wl.offsets.astype(np.int64))
    # chunk 1: nothing is exchanged, the lists keep input order (stable argsort of lengths)
    perm, _ = oracle_mod.oracle_chunks(wl.chars, wl.offsets, 1)
    assert np.array_equal(perm, np.argsort(lens, kind="stable"))
    # one chunk per list: the whole sort
    full, fboff = oracle_mod.oracle_def(wl.chars, wl.offsets)
    perm, boff = oracle_mod.oracle_chunks(wl.chars, wl.offsets, wl.n)
    assert np.array_equal(perm, full) and np.array_equal(boff, fboff)
    # merging the sorted chunks of every list (Python's heapq) gives the whole sort
    import heapq
    words = wl.words()
    for c in (7, 64, 1000):
        perm, boff = oracle_mod.oracle_chunks(wl.chars, wl.offsets, c)
        merged = []
        for L in range(33):
            lo, hi = int(boff[L]), int(boff[L + 1])
            runs = [[(words[i], i) for i in perm[a:min(a + c, hi)]] for a in range(lo, hi, c)]
            for r in runs:
                assert r == sorted(r)
            merged += [i for _, i in heapq.merge(*runs)]
        assert np.array_equal(np.asarray(merged, np.uint32), full), c


def test_parallel_definition_equals_definition(oracle_mod):
    # the per-length-list threads give oracle_def's result: tiny cases (against
    # brute force), empty input, every length, generated text
    for words in list(_tiny_cases())[::7]:
        wl = wordgen.from_words(words)
        exp_perm, exp_boff = brute_force(words)
        perm, boff = oracle_mod.oracle_def_parallel(wl.chars, wl.offsets, threads=3)
        assert np.array_equal(perm, exp_perm) and np.array_equal(boff, exp_boff), words
    perm, boff = oracle_mod.oracle_def_parallel(np.zeros(0, np.uint8), np.zeros(1, np.uint32))
    assert perm.shape[0] == 0 and np.all(boff == 0)
    for cfg, scale in ((1, 1.0), (2, 0.2), (4, 0.002)):
        wl = wordgen.config(cfg, scale)
        p1, b1 = oracle_mod.oracle_def(wl.chars, wl.offsets)
        p2, b2 = oracle_mod.oracle_def_parallel(wl.chars, wl.offsets)
        assert np.array_equal(p1, p2) and np.array_equal(b1, b2)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.oracle_def_parallel(np.zeros(40, np.uint8), np.array([0, 3, 40], np.uint32))
