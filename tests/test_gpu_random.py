"""Randomized GPU parity: many seeded inputs of mixed shape (document counts
and sizes, empty documents, length mixes from all-short to all-long, full
byte range or a tiny alphabet with many equal words), each sorted through
the batched entry point and through a plan with the sorted text, and
compared bit for bit with the oracle's sort and sorted text."""
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


def _random_doc(rng, n):
    mix = int(rng.integers(0, 4))
    if mix == 0:
        lens = rng.integers(0, 33, n)                       # every length
    elif mix == 1:
        lens = np.minimum(1 + rng.geometric(0.3, n), 32)    # mostly short
    elif mix == 2:
        lens = rng.integers(13, 33, n)                      # long words only
    else:
        lens = rng.choice([3, 8, 9, 16, 17], n)             # lane edges
    if rng.integers(0, 2):
        alphabet = np.arange(256, dtype=np.uint8)           # any byte
    else:
        alphabet = np.frombuffer(b"ab", np.uint8)           # many equal words
    return wordgen.from_words([alphabet[rng.integers(0, alphabet.size, L)].tobytes() for L in lens])


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    nd = int(rng.integers(1, 40))
    docs = []
    for _ in range(nd):
        kind = rng.integers(0, 10)
        n = 0 if kind == 0 else int(rng.integers(1, 12) if kind < 3 else rng.integers(100, 20000))
        docs.append(_random_doc(rng, n))
    return wordgen.concat_docs(docs)


@pytest.mark.parametrize("seed", list(range(16)))
def test_random_batches(gpu, oracle_mod, seed):
    import torch
    wl = _case(seed)
    sep = [10, -1, 0, 255][seed % 4]
    _say("case random seed=%d docs=%d n=%d sep=%d" % (seed, wl.n_docs, wl.n, sep))
    eperm, eboff = oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets, fn="oracle_def")
    etext = oracle_mod.oracle_materialize_batch(wl.chars, wl.offsets, wl.doc_offsets, eperm, sep)
    perm, boff = gpu.sort_wordlist(wl)
    assert np.array_equal(perm, eperm) and np.array_equal(boff, eboff), "batch entry point"
    chars, offs, docs = gpu.device_words(wl)
    size = gpu.text_size(wl, sep)
    p2 = torch.empty(max(wl.n, 1), dtype=torch.int32, device="cuda")
    b2 = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
    out = torch.full((size + 32,), 0xAB, dtype=torch.uint8, device="cuda")
    plan = gpu.Plan(wl.n, wl.n_docs)
    try:
        plan.run_text(chars, offs, docs, wl.n_docs, wl.n, p2, b2, sep, out)
        assert plan.status_code() == 0
    finally:
        plan.close()
    o = out.cpu().numpy()
    assert np.array_equal(gpu.to_u32(p2)[:wl.n], eperm), "plan permutation"
    assert np.array_equal(gpu.to_u32(b2).reshape(wl.n_docs, 34), eboff), "plan bucket offsets"
    assert o[:size].tobytes() == etext, "sorted text"
    assert (o[size:] == 0xAB).all(), "bytes past the text"
