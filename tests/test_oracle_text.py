"""Pins of the oracle's text steps around the sort: tokenizing raw text (the
first pre-processing phase, section 3) and writing the sorted words out
(section 4).  Hand-written golden cases, a Python twin built on
``bytes.split`` (ASCII whitespace) and closed forms; CPU only."""
import os

import numpy as np
import pytest

import oracle as orc
from paper_1411_5283_amd import wordgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _unescape(s):
    return s.encode("latin-1").decode("unicode_escape").encode("latin-1")


def _golden(name):
    recs, cur = [], {}
    for line in open(os.path.join(GOLDEN, name), encoding="latin-1"):
        line = line.rstrip("\n")
        if not line or line.startswith("#"):
            continue
        key, _, val = line.partition(": ")
        if key.endswith(":"):          # "text:" with an empty value
            key, val = key[:-1], ""
        cur[key] = val
        if key in ("lower", "sorted"):
            recs.append(cur)
            cur = {}
    return recs


def _words(chars, offs):
    return [chars[offs[i]:offs[i + 1]].tobytes() for i in range(len(offs) - 1)]


def twin_tokenize(text: bytes, lower: bool):
    """Python definition: split on ASCII whitespace, keep ASCII letters."""
    out = []
    for tok in text.split():
        w = bytes(c for c in tok if (65 <= c <= 90) or (97 <= c <= 122))
        if w:
            out.append(w.lower() if lower else w)
    return out


@pytest.mark.parametrize("case", range(5))
def test_tokenize_golden(oracle_mod, case):
    rec = _golden("tokenize_example.txt")[case]
    text = _unescape(rec["text"])
    for flags, key in ((0, "words"), (orc.TOK_LOWER, "lower")):
        want = [] if rec[key] == "-" else [w.encode() for w in rec[key].split(" ")]
        c, o = orc.oracle_tokenize(text, flags)
        assert _words(c, o) == want, (rec, flags)
        assert o[0] == 0 and o[-1] == c.size


def test_tokenize_matches_python_twin(oracle_mod):
    rng = np.random.default_rng(3)
    alphabet = np.frombuffer(b"abcXYZ   \t\n\r\x0b\x0c-'.,0129\x00\xff\xe9", np.uint8)
    for trial in range(300):
        n = int(rng.integers(0, 400))
        if trial % 3 == 0:
            text = rng.integers(0, 256, n, dtype=np.uint8).tobytes()   # every byte value
        else:
            text = alphabet[rng.integers(0, alphabet.size, n)].tobytes()
        for lower in (False, True):
            c, o = orc.oracle_tokenize(text, orc.TOK_LOWER if lower else 0)
            assert _words(c, o) == twin_tokenize(text, lower), text


def test_tokenize_closed_forms(oracle_mod):
    assert _words(*orc.oracle_tokenize(b"")) == []
    assert _words(*orc.oracle_tokenize(b"12 -- ?? \xff")) == []
    assert _words(*orc.oracle_tokenize(b"abcdefXYZ")) == [b"abcdefXYZ"]
    assert _words(*orc.oracle_tokenize(b" ".join([b"w"] * 1000))) == [b"w"] * 1000
    # a text written from a word list with single spaces reads back as that list
    wl = wordgen.single(5000, 800, 1.0, 16, seed=4)
    words = wl.words()
    c, o = orc.oracle_tokenize(b" ".join(words))
    assert _words(c, o) == words
    with pytest.raises(orc.OracleError) as e:
        orc.oracle_tokenize(b"a b c", max_words=2)
    assert e.value.code == orc.CAPACITY


@pytest.mark.parametrize("case", range(3))
def test_materialize_golden(oracle_mod, case):
    rec = _golden("materialize_example.txt")[case]
    words = [w.encode() for w in rec["words"].split(" ")]
    wl = wordgen.from_words(words)
    perm, _ = orc.oracle_def(wl.chars, wl.offsets)
    assert orc.oracle_materialize(wl.chars, wl.offsets, perm, ord("|")) == rec["sorted"].encode()
    assert orc.oracle_materialize(wl.chars, wl.offsets, perm, -1) == rec["sorted"].replace("|", "").encode()


def test_materialize_matches_python_sorted(oracle_mod):
    for seed in range(5):
        wl = wordgen.single(3000, 300, 1.0, 20, seed=seed)
        words = wl.words()
        perm, _ = orc.oracle_bubble(wl.chars, wl.offsets)
        want = b"".join(w + b"\n" for w in sorted(words, key=lambda w: (len(w), w)))
        assert orc.oracle_materialize(wl.chars, wl.offsets, perm, 10) == want


def test_materialize_batch_and_errors(oracle_mod):
    wl = wordgen.concat_docs([wordgen.single(300, 200, 1.0, 12, seed=8), wordgen.from_words([]),
                              wordgen.single(50, 20, 1.0, 6, seed=9), wordgen.from_words([b"x"])])
    perm, _ = orc.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets, "oracle_def")
    got = orc.oracle_materialize_batch(wl.chars, wl.offsets, wl.doc_offsets, perm, 32)
    want = []
    for d in range(wl.n_docs):
        lo, hi = int(wl.doc_offsets[d]), int(wl.doc_offsets[d + 1])
        ws = [wl.chars[wl.offsets[i]:wl.offsets[i + 1]].tobytes() for i in range(lo, hi)]
        want += [w + b" " for w in sorted(ws, key=lambda w: (len(w), w))]
    assert got == b"".join(want)
    wl = wordgen.from_words([b"ab", b"c"])
    with pytest.raises(orc.OracleError):
        orc.oracle_materialize(wl.chars, wl.offsets, np.array([0, 0], np.uint32))
    with pytest.raises(orc.OracleError):
        orc.oracle_materialize(wl.chars, wl.offsets, np.array([0, 2], np.uint32))


# ---------------------------------------------------------------- planted mistakes
_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")
TEXT_MUTANTS = {
    "tok_splits_on_special": ("continue;   /* a special character: removed */",
                              "{ started = 0; continue; }"),
    "tok_keeps_digits": ("return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z');",
                         "return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9');"),
    "tok_no_run_reset": ("            started = 0;\n            continue;", "            continue;"),
    "tok_bad_fold": ("(uint8_t)(c + 32) : c;", "(uint8_t)(c + 31) : c;"),
    "tok_tab_not_space": ("c == ' ' || (c >= 9 && c <= 13)", "c == ' ' || (c >= 10 && c <= 13)"),
    "mat_wrong_source": ("memcpy(out + pos, chars + offsets[i], L);", "memcpy(out + pos, chars + offsets[k], L);"),
    "mat_no_separator": ("out[pos++] = (uint8_t)sep;", "pos++;"),
}


def _mutant_lib(tmp, name):
    import ctypes
    import subprocess
    old, new = TEXT_MUTANTS[name]
    src = open(_SRC).read()
    assert old in src, name
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new, 1))
    so = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", path, "-o", so])
    lib = ctypes.CDLL(so)
    good = orc._load()
    for fn in ("oracle_tokenize", "oracle_materialize", "oracle_def", "oracle_bubble"):
        getattr(lib, fn).argtypes = getattr(good, fn).argtypes
        getattr(lib, fn).restype = getattr(good, fn).restype
    return lib


def _pins_pass():
    try:
        for case in range(5):
            test_tokenize_golden(None, case)
        test_tokenize_matches_python_twin(None)
        for case in range(3):
            test_materialize_golden(None, case)
        test_materialize_matches_python_sorted(None)
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("name", sorted(TEXT_MUTANTS))
def test_text_pins_catch_planted_mistakes(oracle_mod, tmp_path, name):
    lib = _mutant_lib(str(tmp_path), name)
    saved = orc._lib
    orc._lib = lib
    try:
        assert not _pins_pass(), "mutant %s passed every pin" % name
    finally:
        orc._lib = saved
    assert _pins_pass()
