"""GPU parity of sort + sorted text in one pass (sw_plan_run_text): the
permutation and bucket offsets against the oracle's sort, and the text,
written on the device from the sorted keys, byte for byte against the
oracle's sorted text (section 4 prints the merged result) built from the
oracle's own permutation."""
import sys

import numpy as np
import pytest

from paper_1411_5283_amd import wordgen

pytestmark = pytest.mark.gpu

GUARD = 64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1411_5283_amd as sw
    sw.lib()
    torch.cuda.set_device(0)
    return sw


@pytest.fixture
def default_config(gpu):
    cfg = gpu.get_config()
    yield
    gpu.set_config(**cfg)


def _expected(oracle_mod, wl, sep):
    if wl.doc_offsets is None:
        perm, boff = oracle_mod.oracle_def(wl.chars, wl.offsets)
        text = oracle_mod.oracle_materialize(wl.chars, wl.offsets, perm, sep)
    else:
        perm, boff = oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets, fn="oracle_def")
        text = oracle_mod.oracle_materialize_batch(wl.chars, wl.offsets, wl.doc_offsets, perm, sep)
    return perm, boff, text


def _run_text(sw, plan, wl, sep, shift=0):
    """One sw_plan_run_text into a buffer `shift` bytes past an aligned one;
    returns (status, perm, boff, text, guard bytes on both sides untouched)."""
    import torch
    chars, offs, docs = sw.device_words(wl)
    n, nd = wl.n, wl.n_docs
    size = sw.text_size(wl, sep)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    boff = torch.empty(nd * 34, dtype=torch.int32, device="cuda")
    buf = torch.full((shift + size + GUARD,), 0xAB, dtype=torch.uint8, device="cuda")
    plan.run_text(chars, offs, docs, nd, n, perm, boff, sep, buf[shift:])
    st = plan.status_code()
    o = buf.cpu().numpy()
    b = sw.to_u32(boff).reshape(nd, 34)
    guard = bool((o[:shift] == 0xAB).all()) and bool((o[shift + size:] == 0xAB).all())
    return st, sw.to_u32(perm)[:n], (b if docs is not None else b[0]), o[shift:shift + size].tobytes(), guard


def _check(sw, oracle_mod, plan, wl, sep, what, shift=0):
    st, perm, boff, text, guard = _run_text(sw, plan, wl, sep, shift)
    assert st == 0, what
    ep, eb, et = _expected(oracle_mod, wl, sep)
    assert np.array_equal(perm, ep), "%s: permutation differs" % what
    assert np.array_equal(boff, eb), "%s: bucket offsets differ" % what
    assert guard, "%s: bytes written past the text" % what
    if text != et:
        bad = next(k for k in range(len(et)) if text[k] != et[k])
        raise AssertionError("%s: text differs from byte %d of %d" % (what, bad, len(et)))


def _all_lengths(n, seed):
    """Words of every length 0..32 (random bytes), with repeats: every key class,
    the empty word, segments spanning several merge levels."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 33, n)
    vocab = [bytes(rng.integers(0, 256, L, dtype=np.uint8)) for L in lens[: n // 3]]
    pick = rng.integers(0, len(vocab), n)
    return wordgen.from_words([vocab[i] for i in pick])


def _doc_with_segment_sizes(sizes, seed):
    rng = np.random.default_rng(seed)
    words = []
    for L, n in enumerate(sizes, start=1):
        words += [bytes(rng.integers(97, 100, L, dtype=np.uint8)) for _ in range(n)]
    order = rng.permutation(len(words))
    return wordgen.from_words([words[i] for i in order])


@pytest.mark.parametrize("sep", [10, 0, 255, -1])
def test_single_document_every_length(gpu, oracle_mod, sep):
    wl = _all_lengths(200_000, seed=41)
    _say("case text single all lengths n=%d sep=%d" % (wl.n, sep))
    plan = gpu.Plan(wl.n, 1)
    try:
        _check(gpu, oracle_mod, plan, wl, sep, "all lengths sep %d" % sep)
    finally:
        plan.close()


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_output(gpu, oracle_mod, shift):
    # the text is stored as whole dwords of the output's own alignment
    wl = _all_lengths(20_000, seed=43)
    _say("case text unaligned shift=%d n=%d" % (shift, wl.n))
    plan = gpu.Plan(wl.n, 1)
    try:
        for sep in (10, -1):
            _check(gpu, oracle_mod, plan, wl, sep, "shift %d sep %d" % (shift, sep), shift)
    finally:
        plan.close()


def test_zipf_words_many_levels(gpu, oracle_mod):
    wl = wordgen.single(1_500_000, 40_000, 1.1, 24, seed=5)
    _say("case text zipf n=%d" % wl.n)
    plan = gpu.Plan(wl.n, 1)
    try:
        _check(gpu, oracle_mod, plan, wl, 10, "zipf 1.5M")
    finally:
        plan.close()


def test_batch_with_empty_and_tiny_documents(gpu, oracle_mod):
    # one-word and empty documents make many (document, length) pieces per tile
    docs = [wordgen.single(30_000, 2000, 1.1, 20, seed=1), wordgen.from_words([])]
    docs += [wordgen.from_words([b"w%d" % (d % 7)]) for d in range(700)]
    docs += [wordgen.from_words([b""] * 3), wordgen.from_words([]), _all_lengths(5000, seed=2)]
    docs += [_doc_with_segment_sizes([1023, 1024, 1025, 1, 2, 511, 512, 513], seed=3)]
    docs += [_doc_with_segment_sizes([1, 0, 1, 3], seed=10 + d) for d in range(300)]
    wl = wordgen.concat_docs(docs)
    _say("case text batch docs=%d n=%d" % (wl.n_docs, wl.n))
    plan = gpu.Plan(wl.n, wl.n_docs)
    try:
        for sep in (32, -1):
            _check(gpu, oracle_mod, plan, wl, sep, "batch sep %d" % sep)
    finally:
        plan.close()


def test_plan_alternates_sort_and_text(gpu, oracle_mod):
    # both graphs of one plan, inputs of different sizes in turn: the sort
    # alone stays right after text runs, and text runs after plain ones
    import torch
    big = wordgen.config(3, 0.01)
    small = _all_lengths(30_000, seed=9)
    _say("case text alternate big=%d small=%d" % (big.n, small.n))
    plan = gpu.Plan(big.n, big.n_docs)
    try:
        for rep in range(2):
            for wl in (big, small):
                _check(gpu, oracle_mod, plan, wl, 10, "alternate text rep %d n=%d" % (rep, wl.n))
                chars, offs, docs = gpu.device_words(wl)
                perm = torch.empty(max(wl.n, 1), dtype=torch.int32, device="cuda")
                boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
                plan.run(chars, offs, docs, wl.n_docs, wl.n, perm, boff)
                plan.status()
                ep, _, _ = _expected(oracle_mod, wl, 10)
                assert np.array_equal(gpu.to_u32(perm)[:wl.n], ep), "alternate sort rep %d" % rep
    finally:
        plan.close()


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_every_variant(gpu, oracle_mod, default_config, variant):
    wl = wordgen.single(400_000, 30_000, 1.1, 24, seed=7)
    _say("case text variant=%d n=%d" % (variant, wl.n))
    gpu.set_config(chunk=[16, 32, 64, 16, 32],
                   variant=[min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)])
    plan = gpu.Plan(wl.n, 1)
    try:
        _check(gpu, oracle_mod, plan, wl, 10, "variant %d" % variant)
    finally:
        plan.close()


def test_empty_and_one_word(gpu, oracle_mod):
    plan = gpu.Plan(16, 1)
    try:
        for words in ([], [b""], [b"x"], [b"abcdefghijklmnopqrstuvwxyzabcdef"]):
            wl = wordgen.from_words(words)
            _say("case text tiny n=%d" % wl.n)
            _check(gpu, oracle_mod, plan, wl, 10, "tiny %r" % words[:1])
    finally:
        plan.close()


def test_word_too_long_writes_no_text(gpu):
    wl = wordgen.from_words([b"ab", b"c" * 33, b"de"])
    _say("case text too long")
    plan = gpu.Plan(wl.n, 1)
    try:
        st, _, _, text, guard = _run_text(gpu, plan, wl, 10)
        assert st == gpu.ERR_WORD_TOO_LONG
        assert guard and text == b"\xab" * len(text)
    finally:
        plan.close()
