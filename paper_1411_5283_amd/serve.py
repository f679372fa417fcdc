"""Serving loop: continuous batching of word-sort requests on one GPU.

Requests (one document each) arrive at any time.  The scheduler admits them
in arrival order while the device bytes of everything admitted stay within
an HBM budget, packs every admitted request that is not yet running into one
batch, and launches the batch on a free stream as one run of a graph-captured
plan (``sort_words_batch``'s semantics: every (document, length) pair is a
segment).  Batches on different streams overlap on the device.  Completion
is detected with events; then the request's result (its permutation and
bucket offsets, document-local) is handed to its future, its bytes are
released and its latency is recorded.

A request's words stay on the device from its batch's upload until its
batch completes.  A request that can never fit the budget, or that is
malformed (offsets that decrease, a word longer than 32 bytes), fails alone
with the library's error code; the others are unaffected.

The executor is pluggable: ``GpuExecutor`` runs the HIP library; tests use
a CPU stand-in with a simulated clock to check the scheduling rules.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import (ERR_INVALID_ARG, ERR_WORD_TOO_LONG, ERR_WORKSPACE, MAX_LEN, NUM_OFFSETS, SortWordsError,
               decode_status)

HEADER_BYTES = NUM_OFFSETS * 4


def footprint(n_words: int, n_chars: int) -> int:
    """Device bytes a request holds while admitted: its characters, offsets,
    output permutation and bucket offsets."""
    return int(n_chars) + 4 * (int(n_words) + 1) + 4 * int(n_words) + HEADER_BYTES


def check_request(chars: np.ndarray, offsets: np.ndarray) -> int:
    """Host-side argument check of one request (0 or a library error code).
    Works on the uint32 offsets in place (no widening copies)."""
    o = offsets
    if o.ndim != 1 or o.shape[0] < 1:
        return ERR_INVALID_ARG
    if o.shape[0] == 1:
        return 0
    hi, lo = o[1:], o[:-1]
    if (hi < lo).any() or int(o[-1]) > chars.shape[0]:
        return ERR_INVALID_ARG
    if int((hi - lo).max()) > MAX_LEN:
        return ERR_WORD_TOO_LONG
    return 0


@dataclass
class Request:
    rid: int
    chars: np.ndarray
    offsets: np.ndarray          # uint32, rebased so offsets[0] == 0
    arrival: float
    future: Future
    n: int = 0
    bytes: int = 0
    start: float = 0.0
    done: float = 0.0


@dataclass
class Batch:
    requests: list
    handle: object = None
    launched: float = 0.0
    words: int = 0
    docs: int = 0


@dataclass
class Stats:
    completed: int = 0
    failed: int = 0
    words: int = 0
    batches: int = 0
    latencies: list = field(default_factory=list)
    max_bytes_in_use: int = 0

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.asarray(self.latencies), q)) if self.latencies else float("nan")


class SortServer:
    """Continuous-batching scheduler.

    executor: has ``slots`` (concurrent batches), ``launch(batch) -> handle``,
    ``poll(handle) -> bool`` and ``results(handle) -> [(perm, boff), ...]``
    in request order, and ``capacity(words, docs) -> bool``.
    budget_bytes: device bytes all admitted requests may hold together.
    """

    def __init__(self, executor, budget_bytes: int = 8 << 30, max_batch_words: int = 1 << 23,
                 max_batch_docs: int = 1024, min_batch_words: int = 0, max_wait_s: float = 0.0,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch_words = int(max_batch_words)
        self.max_batch_docs = int(max_batch_docs)
        # while another batch is running, a new one starts only once it holds
        # min_batch_words or its oldest request has waited max_wait_s
        self.min_batch_words = int(min_batch_words)
        self.max_wait_s = float(max_wait_s)
        self.clock = clock
        self.queue = collections.deque()      # arrived, not admitted
        self.ready = []                        # admitted, not launched
        self.running = []                      # launched batches
        self.in_use = 0
        self.stats = Stats()
        self._next_id = 0
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._thread = None
        self._stop = False

    # ---------------------------------------------------------------- intake
    def submit(self, chars, offsets) -> Future:
        """Queue one request (host arrays); the future yields (perm, bucket_offsets)."""
        fut = Future()
        chars = np.ascontiguousarray(chars, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
        code = check_request(chars, offsets)
        with self._lock:
            rid = self._next_id
            self._next_id += 1
        if code:
            self.stats.failed += 1
            fut.set_exception(SortWordsError(code, "request %d rejected" % rid))
            return fut
        base = int(offsets[0])
        n = offsets.shape[0] - 1
        req = Request(rid, chars[base:int(offsets[-1])], offsets - np.uint32(base) if base else offsets,
                      self.clock(), fut, n=n)
        req.bytes = footprint(n, req.chars.shape[0])
        if req.bytes > self.budget or n > self.max_batch_words or not self.ex.capacity(n, 1):
            self.stats.failed += 1
            fut.set_exception(SortWordsError(ERR_WORKSPACE, "request %d (%d words) can never fit" % (rid, n)))
            return fut
        with self._wake:
            self.queue.append(req)
            self._wake.notify()
        return fut

    # ---------------------------------------------------------------- scheduling
    def _admit(self):
        """FIFO admission while the budget allows (head-of-line order kept)."""
        while self.queue:
            r = self.queue[0]
            if self.in_use + r.bytes > self.budget:
                break
            self.queue.popleft()
            self.in_use += r.bytes
            self.stats.max_bytes_in_use = max(self.stats.max_bytes_in_use, self.in_use)
            self.ready.append(r)

    def _worth_launching(self) -> bool:
        if not self.running:
            return True
        words = sum(r.n for r in self.ready)
        if words >= self.min_batch_words or len(self.ready) >= self.max_batch_docs:
            return True
        return self.clock() - self.ready[0].arrival >= self.max_wait_s

    def _launch(self):
        while self.ready and len(self.running) < self.ex.slots and self._worth_launching():
            take, words = [], 0
            for r in self.ready:
                if take and (words + r.n > self.max_batch_words or len(take) >= self.max_batch_docs
                             or not self.ex.capacity(words + r.n, len(take) + 1)):
                    break
                take.append(r)
                words += r.n
            self.ready = self.ready[len(take):]
            b = Batch(take, words=words, docs=len(take))
            now = self.clock()
            for r in take:
                r.start = now
            b.launched = now
            try:
                b.handle = self.ex.launch(b)
            except SortWordsError as e:          # the whole batch failed to launch
                self._finish(b, error=e)
                continue
            self.running.append(b)
            self.stats.batches += 1

    def _finish(self, b: Batch, error=None):
        now = self.clock()
        results = None
        if error is None:
            try:
                results = self.ex.results(b.handle)
            except SortWordsError as e:
                error = e
        for i, r in enumerate(b.requests):
            r.done = now
            self.in_use -= r.bytes
            if error is not None:
                self.stats.failed += 1
                r.future.set_exception(error)
            else:
                self.stats.completed += 1
                self.stats.words += r.n
                self.stats.latencies.append(r.done - r.arrival)
                r.future.set_result(results[i])

    def _reap(self) -> bool:
        done = [b for b in self.running if self.ex.poll(b.handle)]
        for b in done:
            self.running.remove(b)
            self._finish(b)
        return bool(done)

    def step(self) -> bool:
        """One scheduler pass: reap finished batches, admit, launch.  Returns
        whether anything is still queued, admitted or running."""
        with self._lock:
            self._reap()
            self._admit()
            self._launch()
            return bool(self.queue or self.ready or self.running)

    def run_until_idle(self, poll_s: float = 0.0):
        while self.step():
            if poll_s:
                time.sleep(poll_s)

    # ---------------------------------------------------------------- background mode
    def start(self, poll_s: float = 50e-6):
        self._stop = False

        def loop():
            while True:
                with self._wake:
                    if self._stop and not (self.queue or self.ready or self.running):
                        return
                    if not (self.queue or self.ready or self.running):
                        self._wake.wait(0.01)
                        continue
                self.step()
                time.sleep(poll_s)

        self._thread = threading.Thread(target=loop, name="sortwords-server", daemon=True)
        self._thread.start()

    def stop(self):
        with self._wake:
            self._stop = True
            self._wake.notify()
        if self._thread:
            self._thread.join()
            self._thread = None


class GpuExecutor:
    """Runs batches on the GPU: one graph-captured plan and one stream per slot.

    Per batch: the requests are packed into one CSR word list in pinned host
    memory, copied to the device on the slot's stream, sorted by the plan,
    and the results copied back; an event marks completion."""

    def __init__(self, slots: int = 2, max_batch_words: int = 1 << 23, max_batch_docs: int = 1024,
                 max_batch_chars: int | None = None, device: str = "cuda"):
        import torch
        from . import Plan
        self.torch = torch
        self.device = torch.device(device)
        self.slots = int(slots)
        self.max_words = int(max_batch_words)
        self.max_docs = int(max_batch_docs)
        self.max_chars = int(max_batch_chars or self.max_words * MAX_LEN)
        self._free = []
        for _ in range(self.slots):
            s = torch.cuda.Stream(device=self.device)
            slot = {
                "stream": s,
                "plan": Plan(self.max_words, self.max_docs, stream=s, max_chars=self.max_chars),
                "chars": torch.empty(max(self.max_chars, 1), dtype=torch.uint8, device=self.device),
                "offsets": torch.empty(self.max_words + 1, dtype=torch.int32, device=self.device),
                "docs": torch.empty(self.max_docs + 1, dtype=torch.int32, device=self.device),
                "perm": torch.empty(max(self.max_words, 1), dtype=torch.int32, device=self.device),
                "boff": torch.empty(self.max_docs * NUM_OFFSETS, dtype=torch.int32, device=self.device),
                "h_chars": torch.empty(max(self.max_chars, 1), dtype=torch.uint8, pin_memory=True),
                "h_offsets": torch.empty(self.max_words + 1, dtype=torch.int32, pin_memory=True),
                "h_docs": torch.empty(self.max_docs + 1, dtype=torch.int32, pin_memory=True),
                "h_perm": torch.empty(max(self.max_words, 1), dtype=torch.int32, pin_memory=True),
                "h_boff": torch.empty(self.max_docs * NUM_OFFSETS, dtype=torch.int32, pin_memory=True),
                "event": torch.cuda.Event(),
                "h_status": torch.zeros(1, dtype=torch.int32, pin_memory=True),
            }
            self._free.append(slot)

    def fixed_bytes(self) -> int:
        from . import sort_words_workspace_size
        per = (sort_words_workspace_size(self.max_words, self.max_docs) + self.max_chars
               + 8 * self.max_words + 4 * self.max_docs * (NUM_OFFSETS + 1))
        return self.slots * per

    def capacity(self, words: int, docs: int) -> bool:
        return words <= self.max_words and docs <= self.max_docs

    def launch(self, batch: Batch):
        torch = self.torch
        if not self._free:
            raise RuntimeError("no free slot")
        slot = self._free.pop()
        reqs = batch.requests
        nchars = sum(r.chars.shape[0] for r in reqs)
        if nchars > self.max_chars:
            self._free.append(slot)
            raise SortWordsError(ERR_WORKSPACE, "batch characters exceed the staging buffer")
        hc = slot["h_chars"].numpy()
        ho = slot["h_offsets"].numpy().view(np.uint32)
        hd = slot["h_docs"].numpy().view(np.uint32)
        c0 = w0 = 0
        ho[0] = 0
        hd[0] = 0
        for d, r in enumerate(reqs):
            nc = r.chars.shape[0]
            hc[c0:c0 + nc] = r.chars
            ho[w0 + 1:w0 + r.n + 1] = r.offsets[1:] + c0
            c0 += nc
            w0 += r.n
            hd[d + 1] = w0
        s = slot["stream"]
        with torch.cuda.stream(s):
            slot["chars"][:max(c0, 1)].copy_(slot["h_chars"][:max(c0, 1)], non_blocking=True)
            slot["offsets"][:w0 + 1].copy_(slot["h_offsets"][:w0 + 1], non_blocking=True)
            slot["docs"][:len(reqs) + 1].copy_(slot["h_docs"][:len(reqs) + 1], non_blocking=True)
            slot["plan"].run(slot["chars"], slot["offsets"], slot["docs"], len(reqs), w0,
                             slot["perm"], slot["boff"])
            slot["h_perm"][:max(w0, 1)].copy_(slot["perm"][:max(w0, 1)], non_blocking=True)
            slot["h_boff"][:len(reqs) * NUM_OFFSETS].copy_(slot["boff"][:len(reqs) * NUM_OFFSETS],
                                                            non_blocking=True)
            slot["plan"].status_async(slot["h_status"])
            slot["event"].record(s)
        return (slot, batch, w0)

    def poll(self, handle) -> bool:
        return handle[0]["event"].query()

    def results(self, handle):
        slot, batch, w0 = handle
        try:
            slot["event"].synchronize()
            code = decode_status(int(slot["h_status"][0]))
            if code != 0:
                raise SortWordsError(code, "batch failed on the device")
            hp = slot["h_perm"].numpy().view(np.uint32)
            hb = slot["h_boff"].numpy().view(np.uint32)
            out, w = [], 0
            for d, r in enumerate(batch.requests):
                out.append((hp[w:w + r.n].copy(), hb[d * NUM_OFFSETS:(d + 1) * NUM_OFFSETS].copy()))
                w += r.n
            return out
        finally:
            self._free.append(slot)

    def close(self):
        for slot in self._free:
            slot["plan"].close()
        self._free = []
