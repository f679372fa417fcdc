"""GPU parity of the steps around the sort, through the C ABI:
sort_words_tokenize (raw text to the word list, section 3's first
pre-processing phase) and sort_words_materialize (the sorted words written
out, section 4), bit for bit against the CPU oracle on the same seeded
inputs, plus the whole chain text -> words -> sort -> sorted text."""
import sys

import numpy as np
import pytest

from paper_1411_5283_amd import wordgen

pytestmark = pytest.mark.gpu

TOK_BLOCK = 256 * 64   # bytes per tokenizer workgroup


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


def _gpu_tokenize(sw, text: bytes, flags=0, max_words=None, shift=0):
    """Tokenize `text` placed `shift` bytes into a device buffer; returns (rc, chars, offsets)."""
    import torch
    n = len(text)
    cap = (n + 1) // 2 if max_words is None else max_words
    buf = torch.zeros(n + shift + 16, dtype=torch.uint8, device="cuda")
    if n:
        buf[shift:shift + n] = torch.from_numpy(np.frombuffer(text, np.uint8).copy()).cuda()
    src = buf[shift:]
    out_chars = torch.full((max(n, 1),), 0xEE, dtype=torch.uint8, device="cuda")
    out_offs = torch.full((cap + 1,), -1, dtype=torch.int32, device="cuda")
    nw = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(sw.tokenize_workspace_size(n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sw.tokenize(src, n, flags, out_chars, out_offs, cap, nw, ws, stream)
    rc = sw.sort_words_status_code(ws, stream)
    if rc:
        return rc, None, None
    k = int(nw.cpu()[0])
    offs = sw.to_u32(out_offs)[:k + 1].copy()
    chars = out_chars.cpu().numpy()[:int(offs[-1])].copy()
    return 0, chars, offs


def _check_tok(sw, oracle_mod, text, flags=0, shift=0, what=""):
    rc, c, o = _gpu_tokenize(sw, text, flags, shift=shift)
    assert rc == 0, what
    ec, eo = oracle_mod.oracle_tokenize(text, flags)
    assert np.array_equal(o, eo), "%s: offsets differ (%d vs %d words)" % (what, len(o) - 1, len(eo) - 1)
    assert np.array_equal(c, ec), "%s: characters differ" % what


def test_tokenize_edge_texts(gpu, oracle_mod):
    cases = {
        "empty": b"",
        "one_letter": b"a",
        "only_specials": b"12-34 ,.; \xff\xfe" * 100,
        "only_spaces": b" \t\n\r\x0b\x0c" * 50,
        "letters_only": b"abcXYZ" * 3000,                          # one word over two workgroups
        "golden": b"The quick brown fox -- it's 3 o'clock!\te-mail: x@y.z\nRe-Enter",
        "every_byte": bytes(range(256)) * 70,
    }
    for name, text in cases.items():
        for flags in (0, gpu.TOK_LOWER):
            _say("case tokenize %s flags=%d n=%d" % (name, flags, len(text)))
            _check_tok(gpu, oracle_mod, text, flags, what=name)


def test_tokenize_block_boundaries(gpu, oracle_mod):
    # a word, or a run of special characters, straddling every kind of boundary
    base = b"x" * (TOK_BLOCK - 3) + b"-'" + b"yz" + b" " + b"." * (2 * TOK_BLOCK + 5) + b"Tail"
    for shift in (0, 1, 3, 15):
        _say("case tokenize boundaries shift=%d" % shift)
        _check_tok(gpu, oracle_mod, base, gpu.TOK_LOWER, shift=shift, what="boundaries shift %d" % shift)
    # letters whose last non-special byte lies several workgroups back
    text = b"a" + b"0" * (3 * TOK_BLOCK) + b"b c" + b"9" * (TOK_BLOCK + 7) + b" d"
    _check_tok(gpu, oracle_mod, text, 0, what="carry across workgroups")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tokenize_random_texts(gpu, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    alphabet = np.frombuffer(b"abcdefghijklmnopqrstuvwxyzABC   \n\t-'.,0", np.uint8)
    n = int(rng.integers(5 * TOK_BLOCK, 9 * TOK_BLOCK))
    text = alphabet[rng.integers(0, alphabet.size, n)].tobytes()
    raw = rng.integers(0, 256, TOK_BLOCK + 321, dtype=np.uint8).tobytes()
    for t, name in ((text, "alphabet"), (raw, "raw bytes")):
        for flags in (0, gpu.TOK_LOWER):
            shift = int(rng.integers(0, 16))
            _say("case tokenize random seed=%d %s n=%d flags=%d shift=%d" % (seed, name, len(t), flags, shift))
            _check_tok(gpu, oracle_mod, t, flags, shift=shift, what="%s seed %d" % (name, seed))


def test_tokenize_rendered_word_list(gpu, oracle_mod):
    wl = wordgen.config(2)
    text = wordgen.render_text(wl, 77).tobytes()
    _say("case tokenize rendered config2 bytes=%d" % len(text))
    rc, c, o = _gpu_tokenize(gpu, text, gpu.TOK_LOWER)
    assert rc == 0
    assert np.array_equal(o, wl.offsets) and np.array_equal(c, wl.chars)


def test_tokenize_capacity_error(gpu):
    _say("case tokenize capacity")
    rc, _, _ = _gpu_tokenize(gpu, b"a b c d e", 0, max_words=4)
    assert rc == -3   # SW_ERR_WORKSPACE
    rc, _, o = _gpu_tokenize(gpu, b"a b c d e", 0, max_words=5)
    assert rc == 0 and len(o) == 6


# ---------------------------------------------------------------- sorted text
def _gpu_materialize(sw, wl, perm, boff, sep, guard=64):
    """Materialize on the device; returns (status word, text bytes, guard bytes untouched)."""
    import torch
    chars, offsets, docs = sw.device_words(wl, "cuda")
    n = wl.n
    size = sw.text_size(wl, sep)
    out = torch.full((size + guard,), 0xAB, dtype=torch.uint8, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    p = torch.from_numpy(np.ascontiguousarray(perm, np.uint32).view(np.int32)).cuda() if n else \
        torch.zeros(1, dtype=torch.int32, device="cuda")
    b = torch.from_numpy(np.ascontiguousarray(boff, np.uint32).reshape(-1).view(np.int32)).cuda()
    nd = wl.n_docs if docs is not None else 1
    sw.materialize(chars, offsets, docs, nd, n, p, b, sep, out, st)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return int(st.cpu()[0]), o[:size].tobytes(), bool((o[size:] == 0xAB).all())


@pytest.mark.parametrize("sep", [10, 32, 0, -1])
def test_materialize_single(gpu, oracle_mod, sep):
    wl = wordgen.single(120_000, 9000, 1.05, 24, seed=12)
    _say("case materialize single n=%d sep=%d" % (wl.n, sep))
    perm, boff = gpu.sort_wordlist(wl)
    st, text, guard = _gpu_materialize(gpu, wl, perm, boff, sep)
    assert st == 0 and guard
    assert text == oracle_mod.oracle_materialize(wl.chars, wl.offsets, perm, sep)


def test_materialize_batch_and_empty_docs(gpu, oracle_mod):
    wl = wordgen.concat_docs([wordgen.single(7000, 600, 1.0, 20, seed=1), wordgen.from_words([]),
                              wordgen.single(1, 5, 1.0, 4, seed=2), wordgen.from_words([b""] * 3),
                              wordgen.single(30_000, 2000, 1.1, 12, seed=3)])
    _say("case materialize batch docs=%d n=%d" % (wl.n_docs, wl.n))
    perm, boff = gpu.sort_wordlist(wl)
    for sep in (10, -1):
        st, text, guard = _gpu_materialize(gpu, wl, perm, boff, sep)
        assert st == 0 and guard
        assert text == oracle_mod.oracle_materialize_batch(wl.chars, wl.offsets, wl.doc_offsets, perm, sep)


def test_materialize_rejects_bad_inputs(gpu, oracle_mod):
    wl = wordgen.single(5000, 400, 1.0, 16, seed=21)
    perm, boff = gpu.sort_wordlist(wl)
    bad_perm = perm.copy()
    bad_perm[17] = wl.n + 5                      # index outside the document
    _say("case materialize bad perm")
    st, _, guard = _gpu_materialize(gpu, wl, bad_perm, boff, 10)
    assert st != 0 and guard
    bad_boff = boff.copy()
    bad_boff[5:] = np.minimum(bad_boff[5:] + 3, wl.n)   # buckets that disagree with the lengths
    _say("case materialize bad bucket offsets")
    st, _, guard = _gpu_materialize(gpu, wl, perm, bad_boff, 10)
    assert st != 0 and guard
    swapped = perm.copy()
    i = int(boff[3])
    j = int(boff[9])
    swapped[i], swapped[j] = swapped[j], swapped[i]    # a 3-letter and a 9-letter word trade places
    st, _, guard = _gpu_materialize(gpu, wl, swapped, boff, -1)
    assert st != 0 and guard


def test_text_sort_text_chain(gpu, oracle_mod):
    # raw text -> word list -> sorted permutation -> sorted text, all on the GPU
    wl = wordgen.single(200_000, 20_000, 1.0, 20, seed=31)
    text = wordgen.render_text(wl, 9).tobytes()
    _say("case chain bytes=%d" % len(text))
    rc, c, o = _gpu_tokenize(gpu, text, gpu.TOK_LOWER)
    assert rc == 0
    got_wl = wordgen.WordList(c, o)
    perm, boff = gpu.sort_wordlist(got_wl)
    st, out, guard = _gpu_materialize(gpu, got_wl, perm, boff, 10)
    assert st == 0 and guard
    ec, eo = oracle_mod.oracle_tokenize(text, oracle_mod.TOK_LOWER)
    eperm, _ = oracle_mod.oracle_def(ec, eo)
    assert out == oracle_mod.oracle_materialize(ec, eo, eperm, 10)


@pytest.mark.parametrize("lower,sep", [(True, 10), (False, 32), (False, -1)])
def test_sort_text_convenience(gpu, oracle_mod, lower, sep):
    # the one-call form (text in, sorted words out) against the oracle's chain
    wl = wordgen.single(120_000, 8_000, 1.0, 24, seed=52)
    text = wordgen.render_text(wl, 3).tobytes()
    _say("case sort_text lower=%s sep=%d bytes=%d" % (lower, sep, len(text)))
    got = gpu.sort_text(text, lower=lower, sep=sep)
    ec, eo = oracle_mod.oracle_tokenize(text, oracle_mod.TOK_LOWER if lower else 0)
    eperm, _ = oracle_mod.oracle_def(ec, eo)
    assert got == oracle_mod.oracle_materialize(ec, eo, eperm, sep)
    assert gpu.sort_text(b"", sep=sep) == b"" and gpu.sort_text(b" \n\t. ,", sep=sep) == b""


def test_sort_strings_convenience(gpu, oracle_mod):
    rng = np.random.default_rng(8)
    words = [bytes(rng.integers(97, 100, int(L), dtype=np.uint8)) for L in rng.integers(0, 33, 5000)]
    words += ["été".encode(), b"\xff\x00", b""]
    got, perm = gpu.sort_strings(words)
    assert got == [w for _, w in sorted(enumerate(words), key=lambda t: (len(t[1]), t[1], t[0]))]
    wl = wordgen.from_words(words)
    eperm, _ = oracle_mod.oracle_def(wl.chars, wl.offsets)
    assert np.array_equal(perm, eperm)
