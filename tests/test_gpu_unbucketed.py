"""GPU parity of the baseline without length lists (sort_words_unbucketed):
one key per word with its length in the top byte, the whole list sorted as
one sequence.  Its result must be the oracle's (the same total order)."""
import sys

import numpy as np
import pytest

from paper_1411_5283_amd import wordgen

pytestmark = pytest.mark.gpu


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


def _run(sw, wl):
    import torch
    chars, offs, _ = sw.device_words(wl, "cuda")
    n = wl.n
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    boff = torch.full((34,), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(sw.sort_words_workspace_size(max(n, 1), 1), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sw.sort_words_unbucketed(chars, offs, n, perm, boff, ws, stream)
    rc = sw.sort_words_status_code(ws, stream)
    return rc, sw.to_u32(perm)[:n], sw.to_u32(boff)


def _random_words(n, seed, max_len=31):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n)
    pool = np.frombuffer(b"\x00\x01abz\x7f\x80\xfe\xff", np.uint8)
    words = []
    for L in lens:
        words.append(pool[rng.integers(0, pool.size, L)].tobytes())
    # duplicates and shared prefixes
    words += [words[i][:max(0, len(words[i]) - 1)] for i in range(0, n, 7)]
    words += words[:n // 5]
    return wordgen.from_words(words)


@pytest.mark.parametrize("case", ["config1", "random_all_lengths", "long_single", "tiny"])
def test_unbucketed_matches_oracle(gpu, oracle_mod, case):
    if case == "config1":
        wl = wordgen.config(1)
    elif case == "random_all_lengths":
        wl = _random_words(40_000, 3)
    elif case == "long_single":
        wl = wordgen.single(600_000, 50_000, 1.1, 24, seed=9)   # many tiles and merge levels
    else:
        wl = wordgen.from_words([b"b", b"", b"a"])
    _say("case unbucketed %s n=%d" % (case, wl.n))
    rc, perm, boff = _run(gpu, wl)
    assert rc == 0
    ep, eb = oracle_mod.oracle_def(wl.chars, wl.offsets)
    bad = np.nonzero(perm != ep)[0]
    assert bad.size == 0, "%s: %d positions differ, first %s" % (case, bad.size, bad[:5])
    assert np.array_equal(boff, eb)


def test_unbucketed_equals_bucketed(gpu):
    wl = wordgen.single(200_000, 20_000, 1.0, 20, seed=4)
    _say("case unbucketed == bucketed n=%d" % wl.n)
    rc, perm, boff = _run(gpu, wl)
    assert rc == 0
    p2, b2 = gpu.sort_wordlist(wl)
    assert np.array_equal(perm, p2) and np.array_equal(boff, b2)


def test_unbucketed_edge_cases(gpu):
    _say("case unbucketed empty")
    rc, perm, boff = _run(gpu, wordgen.from_words([]))
    assert rc == 0 and perm.size == 0 and np.all(boff == 0)
    _say("case unbucketed 31 and 32 bytes")
    rc, perm, _ = _run(gpu, wordgen.from_words([b"z" * 31, b"a" * 31, b"m"]))
    assert rc == 0 and list(perm) == [2, 1, 0]
    rc, _, _ = _run(gpu, wordgen.from_words([b"a", b"q" * 32]))
    assert rc == -2        # SW_ERR_WORD_TOO_LONG: a 32-byte word does not fit the key
    rc, _, _ = _run(gpu, wordgen.from_words([b"a", b"q" * 40]))
    assert rc == -2
    wl = wordgen.from_words([b"ab", b"c"])
    wl.offsets[1], wl.offsets[2] = 3, 2    # offsets that decrease
    rc, _, _ = _run(gpu, wl)
    assert rc == -1
