"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every case sorts through the C ABI (sort_words, sort_words_ex,
sort_words_batch, sort_words_plain, sw_plan_*) and compares the permutation
and the bucket offsets with the oracle on the same seeded input.
"""
import functools
import sys

import numpy as np
import pytest

from checks import check_invariants
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


@pytest.fixture
def default_config(gpu):
    cfg = gpu.get_config()
    yield
    gpu.set_config(**cfg)


def _expect(oracle_mod, wl, bubble=True):
    if wl.doc_offsets is not None:
        return oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets,
                                       fn="oracle_bubble" if bubble else "oracle_def")
    fn = oracle_mod.oracle_bubble if bubble else oracle_mod.oracle_def
    return fn(wl.chars, wl.offsets)


def _same(got, exp, what):
    gp, gb = got
    ep, eb = exp
    assert gp.shape == ep.shape, what
    bad = np.nonzero(gp != ep)[0]
    assert bad.size == 0, "%s: permutation differs at %d positions, first %s" % (what, bad.size, bad[:5])
    assert np.array_equal(gb, eb), "%s: bucket offsets differ" % what


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_long_segments_every_variant(gpu, oracle_mod, default_config, variant):
    # 1.5M words over few lengths: many merge levels and many tiles per workgroup
    wl = wordgen.single(1_500_000, 40_000, 1.1, 20, seed=5)
    _say("case long segments variant=%d n=%d" % (variant, wl.n))
    gpu.set_config(chunk=[16, 32, 64, 16, 32],
                   variant=[min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)])
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "long variant %d" % variant)


@pytest.mark.parametrize("merge", [0, 1, 2])
def test_long_segments_every_merge(gpu, oracle_mod, default_config, merge):
    # the two-way levels (0) and each four-way configuration (1..) of every
    # class, on 1.5M words: many groups, workgroup ranges starting inside
    # groups at every level, short last groups, windows bounded by every run
    wl = wordgen.single(1_500_000, 40_000, 1.1, 20, seed=9)
    m = [min(merge, gpu.num_merges(c) - 1) for c in range(gpu.NUM_CLASSES)]
    _say("case long segments merge=%s n=%d" % (m, wl.n))
    gpu.set_config(merge=m)
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "long merge %s" % m)


@pytest.mark.parametrize("merge", [0, 1, 2])
def test_per_bucket_launch_every_merge(gpu, oracle_mod, default_config, merge):
    # the per-bucket-launch form launches each segment's merge passes directly
    import torch
    wl = wordgen.config(3, 0.01)
    gpu.set_config(merge=[min(merge, gpu.num_merges(c) - 1) for c in range(gpu.NUM_CLASSES)])
    _say("case per-bucket launch merge=%d docs=%d n=%d" % (merge, wl.n_docs, wl.n))
    chars, offs, docs = gpu.device_words(wl)
    ws = torch.empty(gpu.sort_words_workspace_size(wl.n, wl.n_docs), dtype=torch.uint8, device="cuda")
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
    gpu.sort_words_plain(chars, offs, docs, wl.n_docs, perm, boff, ws)
    _same((gpu.to_u32(perm), gpu.to_u32(boff).reshape(wl.n_docs, 34)), _expect(oracle_mod, wl, bubble=False),
          "plain merge %d" % merge)


def test_config1_bit_exact(gpu, oracle_mod):
    wl = wordgen.config(1)
    _say("case config1 n=%d" % wl.n)
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl), "config1")


@pytest.mark.parametrize("variant", [0, 1, 7])
def test_config2_chunk1024_bit_exact(gpu, oracle_mod, default_config, variant):
    # 1024-word odd-even chunks in every class, as configured: variant 0 holds
    # 8 items per thread in classes 2-4 (a chunk spans two waves), variant 1
    # 8 in classes 0-2 and 16 in classes 3-4 (a chunk spans one wave); the
    # short segments' tiles hold 8 per thread; the last variant of every
    # class holds 2 per thread, also in the short segments' tiles (a chunk
    # spans eight waves)
    wl = wordgen.config(2)
    _say("case config2 n=%d chunk=1024 variant=%d" % (wl.n, variant))
    var = [min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)]
    cfg = gpu.set_config(chunk=[1024] * gpu.NUM_CLASSES, variant=var)
    assert cfg["chunk"] == [1024] * gpu.NUM_CLASSES
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "config2")


def _chunk_step_words():
    # a few long lists (several tiles of every variant), short ones, ragged tails
    wl = wordgen.single(70_000, 2500, 1.0, 32, seed=31)
    return wl


CHUNK_WL = None


@pytest.mark.parametrize("chunk", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_chunk_step_bit_exact(gpu, oracle_mod, default_config, chunk, variant):
    # the chunk step alone (odd-even transposition on each chunk of C, no
    # merge) against the oracle's bubble sort of each chunk: every chunk size
    # runs as given, inside a thread, across lanes and across waves
    import torch
    global CHUNK_WL
    if CHUNK_WL is None:
        CHUNK_WL = _chunk_step_words()
    wl = CHUNK_WL
    var = [min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)]
    _say("case chunk step chunk=%d variant=%s n=%d" % (chunk, var, wl.n))
    gpu.set_config(variant=var)
    chars, offs, _ = gpu.device_words(wl, "cuda")
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    boff = torch.empty(34, dtype=torch.int32, device="cuda")
    ws = torch.empty(gpu.sort_words_workspace_size(wl.n, 1), dtype=torch.uint8, device="cuda")
    gpu.sort_words_chunks(chars, offs, wl.n, chunk, perm, boff, ws)
    _same((gpu.to_u32(perm), gpu.to_u32(boff)), oracle_mod.oracle_chunks(wl.chars, wl.offsets, chunk),
          "chunk step %d variant %s" % (chunk, var))


@pytest.mark.parametrize("chunk", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_chunk_and_variant_sweep(gpu, oracle_mod, default_config, chunk, variant):
    # several tiles, merge levels and a ragged tail in every class
    wl = wordgen.single(41_000, 3000, 1.0, 32, seed=77)
    _say("case sweep chunk=%d variant=%d" % (chunk, variant))
    gpu.set_config(chunk=[chunk] * gpu.NUM_CLASSES,
                   variant=[min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)])
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False),
          "chunk %d variant %d" % (chunk, variant))


def _edge_lists():
    rng = np.random.default_rng(11)
    out = {
        "empty": [],
        "one": [b"w"],
        "one_empty_word": [b""],
        "all_empty_words": [b""] * 5000,
        "all_equal": [b"zzz"] * 9000,
        "reversed_distinct": [("%06d" % (99999 - k)).encode() for k in range(12000)],
        "already_sorted": sorted([bytes(rng.integers(97, 123, 6, dtype=np.uint8)) for _ in range(9000)]),
        "all_lengths": [bytes(rng.integers(0, 256, L, dtype=np.uint8)) for L in rng.integers(0, 33, 20000)],
        "unsigned_bytes": [bytes([b]) * L for b in (0, 1, 127, 128, 254, 255) for L in (1, 4, 5, 8, 9, 16, 17, 32)] * 50,
        # words of 0xFF bytes only: the largest keys of every class, in
        # ragged tiles whose slots past the last word hold the fill key just
        # below the sentinel
        "all_ones_ragged": [b"\xff" * L for L in range(33) for _ in range(777)],
        "lane_edges": [bytes(rng.integers(97, 100, L, dtype=np.uint8)) for L in (8, 9, 16, 17, 24, 25, 32) for _ in range(1500)],
        # every word of a length shares all bytes but the last: the order is
        # decided in the class's last lane (lengths 16/17 and 24/25 sit on the
        # edges of the three-lane class)
        "last_byte_decides": [b"p" * (L - 1) + bytes([int(rng.integers(0, 256))])
                              for L in (8, 9, 16, 17, 23, 24, 25, 31, 32) for _ in range(3000)],
    }
    for n in (4095, 4096, 4097, 8193, 2 * 4096 * 4 + 3):
        out["n=%d" % n] = [bytes(rng.integers(97, 99, 3, dtype=np.uint8)) for _ in range(n)]
    return out


EDGES = _edge_lists()


@pytest.mark.parametrize("name", sorted(EDGES))
def test_edge_cases(gpu, oracle_mod, name):
    wl = wordgen.from_words(EDGES[name])
    _say("case edge %s n=%d" % (name, wl.n))
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), name)


SKEWED = ("equal", "reversed", "sawtooth", "sorted", "sorted_every_class")


@functools.lru_cache(maxsize=1)
def _skewed_lists():
    # runs whose key ranges are disjoint or nested after the chunk sort, so
    # that a four-way step is bounded by one run and takes only its window
    # (built when first used: a CPU-only run collects this module too)
    rng = np.random.default_rng(13)
    six = sorted({bytes(rng.integers(97, 123, 6, dtype=np.uint8)) for _ in range(150_000)})
    saw = [b"%07d" % (k % 20_000) for k in range(160_000)]
    by_len = [w for L in (3, 7, 12, 20, 30)
              for w in sorted(bytes(rng.integers(97, 123, L, dtype=np.uint8)) for _ in range(40_000))]
    return {
        "sorted": six,
        "reversed": six[::-1],
        "equal": [b"word"] * 120_000,
        "sawtooth": saw,
        "sorted_every_class": by_len,
    }


@pytest.mark.parametrize("name", SKEWED)
def test_four_way_skewed_runs(gpu, oracle_mod, default_config, name):
    # the four-way passes (every class) against the oracle where the bound of
    # a step comes from one run again and again
    wl = wordgen.from_words(_skewed_lists()[name])
    _say("case four-way skewed %s n=%d" % (name, wl.n))
    gpu.set_config(merge=[1] * gpu.NUM_CLASSES)
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "four-way " + name)


def _three_lane_words(n, seed):
    # lengths 17-24 (three lanes) and 25-26 (four), a shared 16-byte prefix so
    # that lanes 0-1 tie and lane 2 (or 3) decides, plenty of equal words
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.array([17, 18, 20, 23, 24, 25, 26]), n, p=[.3, .15, .15, .1, .2, .05, .05])
    tails = rng.integers(97, 101, (n, 10), dtype=np.uint8)
    return [b"0123456789abcdef" + tails[i, :L - 16].tobytes() for i, L in enumerate(Ls)]


@pytest.mark.parametrize("variant,merge", [(0, 0), (1, 0), (2, 0), (0, 1)])
def test_three_lane_class_long_segments(gpu, oracle_mod, default_config, variant, merge):
    # long segments of the three-lane class: many tiles and merge levels
    # (two-way, or four-way), every tile variant of classes 3 and 4
    wl = wordgen.from_words(_three_lane_words(400_000, 17 + variant))
    _say("case three-lane class variant=%d merge=%d n=%d" % (variant, merge, wl.n))
    gpu.set_config(chunk=[16, 16, 16, 32, 64],
                   variant=[min(variant, gpu.num_variants(c) - 1) for c in range(gpu.NUM_CLASSES)],
                   merge=[min(merge, gpu.num_merges(c) - 1) for c in range(gpu.NUM_CLASSES)])
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "three-lane v%d m%d" % (variant, merge))


def test_nonzero_first_offset_and_unaligned_chars(gpu, oracle_mod):
    import torch
    base = wordgen.config(1, 0.3)
    pad = 3
    chars = np.concatenate([np.full(pad, 7, np.uint8), base.chars])
    offs = (base.offsets + pad).astype(np.uint32)
    _say("case offset0=%d n=%d" % (pad, base.n))
    dchars = torch.from_numpy(chars).cuda()
    doffs = torch.from_numpy(offs.view(np.int32)).cuda()
    perm = torch.empty(base.n, dtype=torch.int32, device="cuda")
    boff = torch.empty(34, dtype=torch.int32, device="cuda")
    gpu.sort_words(dchars, doffs, base.n, perm, boff)
    _same((gpu.to_u32(perm), gpu.to_u32(boff)), oracle_mod.oracle_def(chars, offs), "offset0")


def test_batch_bit_exact(gpu, oracle_mod):
    wl = wordgen.config(3, 0.03)
    _say("case batch docs=%d n=%d" % (wl.n_docs, wl.n))
    got = gpu.sort_wordlist(wl)
    _same(got, _expect(oracle_mod, wl, bubble=False), "batch")


def test_batch_with_empty_docs(gpu, oracle_mod):
    docs = [wordgen.from_words([]), wordgen.config(1, 0.1), wordgen.from_words([]),
            wordgen.from_words([b"b", b"a", b""]), wordgen.config(2, 0.05), wordgen.from_words([])]
    wl = wordgen.concat_docs(docs)
    _say("case batch_empty_docs n=%d" % wl.n)
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl), "batch empty docs")


def test_plain_form_equals_batched(gpu, oracle_mod):
    import torch
    wl = wordgen.config(3, 0.01)
    _say("case plain-vs-batch docs=%d n=%d" % (wl.n_docs, wl.n))
    chars, offs, docs = gpu.device_words(wl)
    ws = torch.empty(gpu.sort_words_workspace_size(wl.n, wl.n_docs), dtype=torch.uint8, device="cuda")
    outs = []
    for fn in (gpu.sort_words_plain, gpu.sort_words_batch):
        perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
        boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
        fn(chars, offs, docs, wl.n_docs, perm, boff, ws)
        gpu.sort_words_status(ws)
        outs.append((gpu.to_u32(perm), gpu.to_u32(boff).reshape(wl.n_docs, 34)))
    _same(outs[0], outs[1], "plain vs batch")
    _same(outs[1], _expect(oracle_mod, wl, bubble=False), "batch vs oracle")


def test_plan_graph_replays(gpu, oracle_mod):
    import torch
    big = wordgen.config(3, 0.02)
    small = wordgen.config(1, 0.5)
    _say("case plan big=%d small=%d" % (big.n, small.n))
    plan = gpu.Plan(big.n, big.n_docs)
    try:
        for rep in range(3):
            for wl in (big, small):
                chars, offs, docs = gpu.device_words(wl)
                perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
                boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
                plan.run(chars, offs, docs, wl.n_docs, wl.n, perm, boff)
                plan.status()
                got = (gpu.to_u32(perm), gpu.to_u32(boff).reshape(wl.n_docs, 34))
                if docs is None:
                    got = (got[0], got[1][0])
                _same(got, _expect(oracle_mod, wl, bubble=False), "plan rep %d n=%d" % (rep, wl.n))
                torch.cuda.synchronize()
    finally:
        plan.close()


def test_device_detected_errors(gpu):
    import torch
    _say("case errors")
    n = 3
    perm = torch.empty(8, dtype=torch.int32, device="cuda")
    boff = torch.empty(34 * 4, dtype=torch.int32, device="cuda")
    chars = torch.zeros(100, dtype=torch.uint8, device="cuda")

    def run(offs):
        o = torch.tensor(np.asarray(offs, np.uint32).view(np.int32), device="cuda")
        try:
            gpu.sort_words(chars, o, len(offs) - 1, perm, boff)
            return 0
        except gpu.SortWordsError as e:
            return e.code

    assert run([0, 3, 40, 41]) == gpu.ERR_WORD_TOO_LONG
    assert run([0, 5, 3, 9]) == gpu.ERR_INVALID_ARG
    assert run([0, 50, 40, 99]) == gpu.ERR_INVALID_ARG      # decreasing beats too long
    assert run([0, 32, 64, 96]) == gpu.OK
    # batch: doc_offsets must start at 0 and not decrease; N above capacity
    o = torch.tensor(np.arange(0, 10, 2, dtype=np.uint32).view(np.int32), device="cuda")
    ws = torch.empty(gpu.sort_words_workspace_size(4, 2), dtype=torch.uint8, device="cuda")
    for docs, code in (([1, 4], gpu.ERR_INVALID_ARG), ([0, 3, 2], gpu.ERR_INVALID_ARG),
                       ([0, 4], gpu.OK)):
        d = torch.tensor(np.asarray(docs, np.uint32).view(np.int32), device="cuda")
        gpu.sort_words_batch(chars, o, d, len(docs) - 1, perm, boff, ws)
        assert gpu.sort_words_status_code(ws) == code, docs
    # 100 words in a workspace sized for 10: the device sees N above capacity
    o100 = torch.tensor(np.arange(0, 101, dtype=np.uint32).view(np.int32), device="cuda")
    perm100 = torch.empty(100, dtype=torch.int32, device="cuda")
    ws_small = torch.empty(gpu.sort_words_workspace_size(10, 1), dtype=torch.uint8, device="cuda")
    d = torch.tensor(np.asarray([0, 100], np.uint32).view(np.int32), device="cuda")
    gpu.sort_words_batch(chars, o100, d, 1, perm100, boff, ws_small)
    assert gpu.sort_words_status_code(ws_small) == gpu.ERR_WORKSPACE
    # a plan made for 200 characters: ten words of 30 bytes (300 characters)
    # are SW_ERR_WORKSPACE, six (180, starting at byte 150) sort
    plan = gpu.Plan(64, 1, max_chars=200)
    big_chars = torch.zeros(400, dtype=torch.uint8, device="cuda")
    try:
        for offs_np, code in ((np.arange(0, 301, 30), gpu.ERR_WORKSPACE), (np.arange(150, 331, 30), gpu.OK)):
            o = torch.tensor(offs_np.astype(np.uint32).view(np.int32), device="cuda")
            nw = len(offs_np) - 1
            plan.run(big_chars, o, None, 1, nw, perm100, boff)
            assert plan.status_code() == code, offs_np
    finally:
        plan.close()
    # after errors the library still sorts correctly
    wl = wordgen.from_words([b"b", b"a"])
    p, b = gpu.sort_wordlist(wl)
    assert list(p) == [1, 0]


def _doc_with_segment_sizes(sizes, seed):
    """A document whose length-L bucket has sizes[L-1] words (random bytes)."""
    rng = np.random.default_rng(seed)
    words = []
    for L, n in enumerate(sizes, start=1):
        words += [bytes(rng.integers(97, 100, L, dtype=np.uint8)) for _ in range(n)]
    order = rng.permutation(len(words))
    return wordgen.from_words([words[i] for i in order])


def test_packed_short_segments(gpu, oracle_mod):
    # segment sizes around the packing threshold (1024) and many one-word segments
    docs = [_doc_with_segment_sizes([1023, 1024, 1025, 1, 2, 511, 512, 513], seed=1),
            _doc_with_segment_sizes([1] * 24, seed=2)]
    docs += [_doc_with_segment_sizes([1, 0, 1, 3], seed=10 + d) for d in range(1500)]
    docs += [_doc_with_segment_sizes([700, 300, 1024, 4], seed=3)]
    wl = wordgen.concat_docs(docs)
    _say("case packed segments docs=%d n=%d" % (wl.n_docs, wl.n))
    _same(gpu.sort_wordlist(wl), _expect(oracle_mod, wl, bubble=False), "packed")


@pytest.mark.parametrize("flags", [0, 2, 4, 6])
def test_short_segment_order_flag(gpu, oracle_mod, default_config, flags):
    # the short-segment sort enqueued after (0) or before (FLAG_PACKED_FIRST)
    # each class's chunk sort, the segment scheduling before or beside
    # (FLAG_SCHEDULE_BESIDE_SCATTER) the scatter: the same result, eager and
    # replayed in a plan
    import torch
    docs = [wordgen.config(1, 0.1), _doc_with_segment_sizes([1023, 1024, 1025, 5, 2048], seed=4)]
    docs += [_doc_with_segment_sizes([1, 0, 1, 3], seed=20 + d) for d in range(300)]
    docs += [wordgen.config(2, 0.05)]
    wl = wordgen.concat_docs(docs)
    _say("case short-segment order flags=%d docs=%d n=%d" % (flags, wl.n_docs, wl.n))
    assert gpu.FLAG_PACKED_FIRST == 2 and gpu.FLAG_SCHEDULE_BESIDE_SCATTER == 4
    gpu.set_config(flags=flags)
    exp = _expect(oracle_mod, wl, bubble=False)
    _same(gpu.sort_wordlist(wl), exp, "flags %d eager" % flags)
    chars, offs, ddocs = gpu.device_words(wl)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
    plan = gpu.Plan(wl.n, wl.n_docs)
    try:
        for rep in range(2):
            plan.run(chars, offs, ddocs, wl.n_docs, wl.n, perm, boff)
            plan.status()
            _same((gpu.to_u32(perm), gpu.to_u32(boff).reshape(wl.n_docs, 34)), exp,
                  "flags %d plan replay %d" % (flags, rep))
    finally:
        plan.close()


def test_every_class_order(gpu, oracle_mod, default_config):
    # the 120 enqueue orders of the classes (with both launch-order flags and
    # without): the same result, eager and in a plan
    import torch
    docs = [wordgen.config(1, 0.1), _doc_with_segment_sizes([1023, 1024, 1025, 5, 2048], seed=5)]
    docs += [_doc_with_segment_sizes([1, 0, 1, 3], seed=40 + d) for d in range(100)]
    wl = wordgen.concat_docs(docs)
    exp = _expect(oracle_mod, wl, bubble=False)
    chars, offs, ddocs = gpu.device_words(wl)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
    for k in range(gpu.NUM_ORDERS):
        flags = (k << gpu.FLAG_ORDER_SHIFT) | (6 if k % 2 else 0)
        _say("case class order %d flags=%d n=%d" % (k, flags, wl.n))
        gpu.set_config(flags=flags)
        _same(gpu.sort_wordlist(wl), exp, "order %d eager" % k)
        plan = gpu.Plan(wl.n, wl.n_docs)
        try:
            plan.run(chars, offs, ddocs, wl.n_docs, wl.n, perm, boff)
            plan.status()
            _same((gpu.to_u32(perm), gpu.to_u32(boff).reshape(wl.n_docs, 34)), exp, "order %d plan" % k)
        finally:
            plan.close()
