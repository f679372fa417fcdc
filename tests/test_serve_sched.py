"""Scheduling rules of the serving loop, on the CPU.

A fake executor stands in for the GPU: it "runs" a batch for a simulated
time and answers with the oracle.  The clock is simulated, so admission,
overlap and latency are deterministic.
"""
import numpy as np
import pytest

from paper_1411_5283_amd import ERR_INVALID_ARG, ERR_WORD_TOO_LONG, ERR_WORKSPACE, SortWordsError, wordgen
from paper_1411_5283_amd.serve import SortServer, footprint


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    def __init__(self, oracle_mod, clock, slots=2, us_per_word=0.01, fail_on=None):
        self.oracle = oracle_mod
        self.clock = clock
        self.slots = slots
        self.us_per_word = us_per_word
        self.fail_on = fail_on or set()
        self.launches = []          # (time, [request ids]) in launch order
        self.active = 0
        self.max_active = 0

    def capacity(self, words, docs):
        return words <= 10_000_000 and docs <= 64

    def launch(self, batch):
        self.launches.append((self.clock(), [r.rid for r in batch.requests]))
        self.active += 1
        self.max_active = max(self.max_active, self.active)
        return {"batch": batch, "done": self.clock() + 1e-6 * self.us_per_word * max(batch.words, 1)}

    def poll(self, h):
        if self.clock() >= h["done"]:
            if not h.get("reaped"):
                h["reaped"] = True
                self.active -= 1
            return True
        return False

    def results(self, h):
        if any(r.rid in self.fail_on for r in h["batch"].requests):
            raise SortWordsError(-5, "simulated device failure")
        return [self.oracle.oracle_def(r.chars, r.offsets) for r in h["batch"].requests]


def _drive(server, clock, dt=1e-4, limit=100000):
    for _ in range(limit):
        if not server.step():
            return
        clock.t += dt
    raise AssertionError("server did not drain")


def _reqs(n, seed=0):
    return [wordgen.config(1, s) for s in np.linspace(0.01, 0.2, n)]


def test_results_match_oracle_and_budget_holds(oracle_mod):
    clock = SimClock()
    ex = FakeExecutor(oracle_mod, clock)
    reqs = _reqs(12)
    budget = 3 * max(footprint(r.n, r.chars.shape[0]) for r in reqs)
    srv = SortServer(ex, budget_bytes=budget, clock=clock)
    futs = [srv.submit(r.chars, r.offsets) for r in reqs]
    _drive(srv, clock)
    for r, f in zip(reqs, futs):
        p, b = f.result()
        ep, eb = oracle_mod.oracle_bubble(r.chars, r.offsets)
        assert np.array_equal(p, ep) and np.array_equal(b, eb)
    assert srv.stats.max_bytes_in_use <= budget
    assert srv.stats.completed == len(reqs) and srv.in_use == 0


def test_fifo_admission(oracle_mod):
    clock = SimClock()
    ex = FakeExecutor(oracle_mod, clock, slots=1)
    reqs = _reqs(10)
    budget = 2 * max(footprint(r.n, r.chars.shape[0]) for r in reqs)
    srv = SortServer(ex, budget_bytes=budget, clock=clock)
    for r in reqs:
        srv.submit(r.chars, r.offsets)
    _drive(srv, clock)
    order = [rid for _, ids in ex.launches for rid in ids]
    assert order == sorted(order) == list(range(len(reqs)))


def test_over_budget_and_malformed_requests_fail_alone(oracle_mod):
    clock = SimClock()
    ex = FakeExecutor(oracle_mod, clock)
    good = _reqs(4)
    budget = 2 * max(footprint(r.n, r.chars.shape[0]) for r in good)
    srv = SortServer(ex, budget_bytes=budget, clock=clock)
    big = wordgen.config(1, 1.0)
    long_word = wordgen.from_words([b"ok", b"x" * 33])
    bad_offsets = (np.zeros(4, np.uint8), np.array([0, 3, 1, 4], np.uint32))
    futs = [srv.submit(good[0].chars, good[0].offsets),
            srv.submit(big.chars, big.offsets),
            srv.submit(long_word.chars, long_word.offsets),
            srv.submit(*bad_offsets),
            srv.submit(good[1].chars, good[1].offsets)]
    _drive(srv, clock)
    codes = []
    for f in futs:
        e = f.exception()
        codes.append(0 if e is None else e.code)
    assert codes == [0, ERR_WORKSPACE, ERR_WORD_TOO_LONG, ERR_INVALID_ARG, 0]


def test_device_failure_fails_only_its_batch(oracle_mod):
    clock = SimClock()
    reqs = _reqs(6)
    ex = FakeExecutor(oracle_mod, clock, slots=1, fail_on={2})
    srv = SortServer(ex, budget_bytes=1 << 30, max_batch_docs=1, clock=clock)   # one request per batch
    futs = [srv.submit(r.chars, r.offsets) for r in reqs]
    _drive(srv, clock)
    failed = [i for i, f in enumerate(futs) if f.exception() is not None]
    assert failed == [2]
    assert srv.in_use == 0


def test_continuous_batching_overlaps(oracle_mod):
    """Requests that arrive while a batch runs are launched on a free slot
    before that batch completes."""
    clock = SimClock()
    ex = FakeExecutor(oracle_mod, clock, slots=2, us_per_word=1.0)
    reqs = _reqs(6)
    srv = SortServer(ex, budget_bytes=1 << 30, clock=clock)
    srv.submit(reqs[0].chars, reqs[0].offsets)
    srv.step()                                   # batch 1 launched
    clock.t += 1e-4
    for r in reqs[1:]:
        srv.submit(r.chars, r.offsets)
    srv.step()                                   # batch 2 launched while 1 runs
    assert len(ex.launches) == 2 and ex.max_active == 2
    _drive(srv, clock)
    assert srv.stats.completed == 6
    lat = srv.stats.latencies
    assert len(lat) == 6 and min(lat) > 0


def test_batching_policy_waits_for_work_or_age(oracle_mod):
    """With a batch running, small arrivals are held until they reach
    min_batch_words or the oldest has waited max_wait_s."""
    clock = SimClock()
    ex = FakeExecutor(oracle_mod, clock, slots=2, us_per_word=100.0)
    reqs = _reqs(5)
    srv = SortServer(ex, budget_bytes=1 << 30, min_batch_words=10 ** 9, max_wait_s=1e-3, clock=clock)
    srv.submit(reqs[0].chars, reqs[0].offsets)
    srv.step()
    assert len(ex.launches) == 1                     # idle GPU: launch at once
    srv.submit(reqs[1].chars, reqs[1].offsets)
    clock.t += 5e-4
    srv.step()
    assert len(ex.launches) == 1                     # too small, too young
    clock.t += 6e-4
    srv.step()
    assert len(ex.launches) == 2                     # aged past max_wait_s
    _drive(srv, clock)
    assert srv.stats.completed == 2
