"""GPU tests of the library's native serving loop (sw_server_*): every
request's result equals the oracle's and the result of sorting it alone;
malformed and oversized requests are refused alone; the HBM budget holds
and binds on the device pool requests wait in;
two client threads submit at once."""
import sys
import threading

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


def _requests(k, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(k):
        n = int(rng.choice([0, 1, 7, 500, 4097, 30_000, 120_000]))
        wl = wordgen.single(max(n, 1), 3000, 1.0, 20, seed=seed * 100 + r)
        if n == 0:
            wl = wordgen.from_words([])
        out.append(wl)
    return out


def test_native_server_results_match_oracle(gpu, oracle_mod):
    reqs = _requests(40, 1)
    _say("case native server mix of %d requests" % len(reqs))
    srv = gpu.NativeServer(slots=2, max_batch_words=1 << 20, max_batch_docs=16, min_batch_words=50_000,
                           max_wait_us=200, copy_threads=3)
    try:
        tickets = [srv.submit(w.chars, w.offsets) for w in reqs]
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["batches"] < len(reqs)
    for w, (perm, boff, lat) in zip(reqs, results):
        ep, eb = oracle_mod.oracle_def(w.chars, w.offsets)
        assert np.array_equal(perm, ep) and np.array_equal(boff, eb)
        assert lat > 0
    # the same requests sorted one at a time give the same results
    for w, (perm, boff, _) in list(zip(reqs, results))[:8]:
        if w.n:
            p2, b2 = gpu.sort_wordlist(w)
            assert np.array_equal(perm, p2) and np.array_equal(boff, b2)


def test_native_server_refuses_bad_requests_alone(gpu, oracle_mod):
    good = wordgen.single(2000, 300, 1.0, 12, seed=7)
    dec = wordgen.from_words([b"ab", b"c", b"d"])
    dec.offsets[2] = 1
    long_ = wordgen.from_words([b"a", b"x" * 33])
    srv = gpu.NativeServer(slots=1, max_batch_words=10_000, max_batch_docs=4, budget_bytes=1 << 20)
    try:
        t1 = srv.submit(good.chars, good.offsets)
        with pytest.raises(gpu.SortWordsError) as e:
            srv.submit(dec.chars, dec.offsets)
        assert e.value.code == gpu.ERR_INVALID_ARG
        with pytest.raises(gpu.SortWordsError) as e:
            srv.submit(long_.chars, long_.offsets)
        assert e.value.code == gpu.ERR_WORD_TOO_LONG
        big = wordgen.single(20_000, 300, 1.0, 12, seed=8)      # larger than a batch
        with pytest.raises(gpu.SortWordsError) as e:
            srv.submit(big.chars, big.offsets)
        assert e.value.code == gpu.ERR_WORKSPACE
        t2 = srv.submit(good.chars, good.offsets)
        for t in (t1, t2):
            perm, boff, _ = srv.wait(t)
            ep, eb = oracle_mod.oracle_def(good.chars, good.offsets)
            assert np.array_equal(perm, ep) and np.array_equal(boff, eb)
    finally:
        srv.close()


def test_native_server_budget_and_slices(gpu, oracle_mod):
    # a budget that holds about three requests: admission must wait for
    # completions, and the budget is never exceeded
    reqs = [wordgen.single(40_000, 5000, 1.0, 16, seed=20 + r) for r in range(12)]
    per = max(gpu.NativeServer.request_bytes(w.n, int(w.offsets[-1] - w.offsets[0])) for w in reqs)
    budget = int(3 * per)
    # requests given as slices of a bigger buffer (first offset not 0)
    big = wordgen.concat_docs(reqs)
    srv = gpu.NativeServer(slots=2, max_batch_words=200_000, max_batch_docs=8, budget_bytes=budget)
    try:
        tickets = []
        for d in range(len(reqs)):
            lo, hi = int(big.doc_offsets[d]), int(big.doc_offsets[d + 1])
            tickets.append(srv.submit(big.chars, big.offsets[lo:hi + 1]))
        out = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert st["max_bytes_in_use"] <= budget and st["completed"] == len(reqs)
    for w, (perm, boff, _) in zip(reqs, out):
        ep, eb = oracle_mod.oracle_def(w.chars, w.offsets)
        assert np.array_equal(perm, ep) and np.array_equal(boff, eb)


def test_native_server_two_client_threads(gpu, oracle_mod):
    reqs = _requests(30, 3)
    srv = gpu.NativeServer(slots=2, max_batch_words=1 << 20, max_batch_docs=32, copy_threads=2)
    got = {}
    lock = threading.Lock()

    def client(part):
        mine = [(i, srv.submit(reqs[i].chars, reqs[i].offsets)) for i in range(part, len(reqs), 2)]
        for i, t in mine:
            r = srv.wait(t)
            with lock:
                got[i] = r
    try:
        th = [threading.Thread(target=client, args=(p,)) for p in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    finally:
        srv.close()
    assert len(got) == len(reqs)
    for i, w in enumerate(reqs):
        ep, eb = oracle_mod.oracle_def(w.chars, w.offsets)
        assert np.array_equal(got[i][0], ep) and np.array_equal(got[i][1], eb)


def test_native_server_budget_binds_on_device_memory(gpu, oracle_mod):
    # requests wait in blocks of a device pool as large as the budget: a
    # budget of 1.5 times the largest request, requests of very mixed sizes
    # (one larger than a staging buffer, so its upload goes in pieces, and
    # empty ones) submitted at once; the pool fills and fragments, admission
    # waits for completions, the budget holds and every result is exact
    rng = np.random.default_rng(44)
    sizes = [700_000, 0, 1, 90_000] + [int(rng.choice([5, 3000, 60_000, 250_000])) for _ in range(36)]
    reqs = [wordgen.single(n, 4000, 1.0, 24, seed=300 + i) if n else wordgen.from_words([])
            for i, n in enumerate(sizes)]
    fp = [gpu.NativeServer.request_bytes(w.n, int(w.offsets[-1] - w.offsets[0])) for w in reqs]
    budget = int(1.5 * max(fp))
    assert sum(fp) > 3 * budget
    _say("case native server binding budget %d bytes, %d requests" % (budget, len(reqs)))
    srv = gpu.NativeServer(slots=2, max_batch_words=1 << 20, max_batch_docs=8, budget_bytes=budget,
                           copy_threads=0)
    try:
        too_big = wordgen.single(int(budget / 4), 4000, 1.0, 24, seed=9)   # more bytes than the budget
        with pytest.raises(gpu.SortWordsError) as e:
            srv.submit(too_big.chars, too_big.offsets)
        assert e.value.code == gpu.ERR_WORKSPACE
        tickets = [srv.submit(w.chars, w.offsets) for w in reqs]
        out = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert max(fp) <= st["max_bytes_in_use"] <= budget and st["bytes_in_use"] == 0
    for w, (perm, boff, _) in zip(reqs, out):
        ep, eb = oracle_mod.oracle_def(w.chars, w.offsets)
        assert np.array_equal(perm, ep) and np.array_equal(boff, eb)


def test_native_server_stress_tight_budget(gpu, oracle_mod):
    # many requests of mixed sizes through a pool of three times the largest
    # request, three slots and four upload threads (uploads grouped where
    # blocks lie back to back), from two client threads at once: the pool
    # fills, fragments and drains many times; every result is exact
    rng = np.random.default_rng(77)
    sizes = np.clip(np.round(rng.lognormal(np.log(2000), 1.2, 300)), 0, 150_000).astype(int)
    reqs = [wordgen.single(int(n), 3000, 1.0, 24, seed=900 + i) if n else wordgen.from_words([])
            for i, n in enumerate(sizes)]
    fp = [gpu.NativeServer.request_bytes(w.n, int(w.offsets[-1] - w.offsets[0])) for w in reqs]
    budget = 3 * max(fp)
    _say("case native server stress: %d requests, %d words, budget %d" % (len(reqs), int(sizes.sum()), budget))
    srv = gpu.NativeServer(slots=3, max_batch_words=1 << 19, max_batch_docs=16, budget_bytes=budget,
                           min_batch_words=20_000, max_wait_us=100, copy_threads=4)
    got = {}
    lock = threading.Lock()

    def client(part):
        mine = []
        for i in range(part, len(reqs), 2):
            mine.append((i, srv.submit(reqs[i].chars, reqs[i].offsets)))
        for i, t in mine:
            r = srv.wait(t)
            with lock:
                got[i] = r
    try:
        th = [threading.Thread(target=client, args=(p,)) for p in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        st = srv.stats()
    finally:
        srv.close()
    assert len(got) == len(reqs) and st["failed"] == 0
    assert st["max_bytes_in_use"] <= budget and st["bytes_in_use"] == 0
    for i, w in enumerate(reqs):
        ep, eb = oracle_mod.oracle_def(w.chars, w.offsets)
        assert np.array_equal(got[i][0], ep) and np.array_equal(got[i][1], eb), i
