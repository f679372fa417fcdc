"""Seeded synthetic word lists: the inputs of the word sort, and nothing else.

This module draws inputs only; it holds none of the sort's arithmetic (no
length bucketing, no comparison, no ordering).  Both the HIP path and the CPU
oracle are fed from it, and it imports neither.

The paper measures on two English texts (Hamlet, 190 KB and 1.38 MB; section
"3. Methodology").  They are not available here, so these generators stand in
for them with English-like statistics:

* vocabulary entry length  l = 1 + G1 + G2,  G ~ Geometric on {0,1,...} with
  success probability 4/11 (mean 4.5 before truncation), redrawn until it lies
  in [1, max_len];  letters i.i.d. uniform over 'a'..'z';
* tokens: Zipf(s) rank over the vocabulary, sampled by inverse CDF.

A word list is CSR: ``chars`` (uint8, no separators) and ``offsets`` (uint32,
n+1 entries); word i is ``chars[offsets[i]:offsets[i+1]]``.  Batches add
``doc_offsets`` (uint32, n_docs+1 entries into the word list).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GEO_P = 4.0 / 11.0
SEED_BASE = 14115283 * 10          # per-config seed = SEED_BASE + config number
DOC_SEED_STRIDE = 1000             # per-document token stream: + 1000 * (doc + 1)
REQUEST_SEED_STRIDE = 10 ** 6      # per-request token stream: + 10**6 * (request + 1)
_CHUNK = 1 << 22                   # tokens per gather step (bounds temporaries)


@dataclass
class WordList:
    chars: np.ndarray                  # uint8 [sum of lengths]
    offsets: np.ndarray                # uint32 [n + 1]
    doc_offsets: np.ndarray | None = None   # uint32 [n_docs + 1] or None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_docs(self) -> int:
        return 1 if self.doc_offsets is None else int(self.doc_offsets.shape[0] - 1)

    def words(self, lo: int = 0, hi: int | None = None) -> list[bytes]:
        hi = self.n if hi is None else hi
        c = self.chars
        o = self.offsets
        return [c[o[i]:o[i + 1]].tobytes() for i in range(lo, hi)]


@dataclass
class Vocabulary:
    chars: np.ndarray      # uint8, concatenated entries
    offsets: np.ndarray    # int64 [V + 1]
    cdf: np.ndarray        # float64 [V], Zipf cumulative distribution over ranks


def make_vocabulary(rng: np.random.Generator, V: int, max_len: int, s: float) -> Vocabulary:
    lens = np.empty(V, np.int64)
    fill = 0
    while fill < V:
        k = V - fill
        l = 1 + (rng.geometric(GEO_P, size=k) - 1) + (rng.geometric(GEO_P, size=k) - 1)
        l = l[(l >= 1) & (l <= max_len)]
        lens[fill:fill + l.shape[0]] = l
        fill += l.shape[0]
    offs = np.zeros(V + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    chars = rng.integers(ord("a"), ord("z") + 1, size=int(offs[-1]), dtype=np.uint8)
    w = np.arange(1, V + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return Vocabulary(chars, offs, cdf)


def draw_tokens(rng: np.random.Generator, vocab: Vocabulary, n: int) -> np.ndarray:
    u = rng.random(n)
    t = np.searchsorted(vocab.cdf, u, side="right")
    np.minimum(t, vocab.cdf.shape[0] - 1, out=t)
    return t


def materialize(vocab: Vocabulary, tokens: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Token ids -> CSR (chars, offsets)."""
    vo = vocab.offsets
    lens = (vo[tokens + 1] - vo[tokens]).astype(np.int64)
    offsets = np.zeros(tokens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    if total >= 1 << 32:
        raise ValueError("word list exceeds 2**32 characters")
    chars = np.empty(total, np.uint8)
    for lo in range(0, tokens.shape[0], _CHUNK):
        hi = min(lo + _CHUNK, tokens.shape[0])
        l = lens[lo:hi]
        dst0 = int(offsets[lo])
        dst1 = int(offsets[hi])
        src = np.repeat(vo[tokens[lo:hi]] - (offsets[lo:hi] - dst0), l)
        src += np.arange(dst1 - dst0, dtype=np.int64)
        chars[dst0:dst1] = vocab.chars[src]
    return chars, offsets.astype(np.uint32)


# --------------------------------------------------------------------------- configs
# Sizes follow the paper's two texts (about 35k and 250k words at ~5.5 bytes per
# word including one separator) and the larger batched / single / serving
# workloads this library is measured on.
CONFIGS = {
    1: dict(kind="single", n=35_000, V=5_000, s=1.0, max_len=16),
    2: dict(kind="single", n=250_000, V=20_000, s=1.0, max_len=20, chunk=1024),
    3: dict(kind="batch", n_docs=4096, doc_min=100, doc_max=50_000, V=50_000, s=1.1, max_len=20),
    4: dict(kind="single", n=64_000_000, V=1_000_000, s=1.1, max_len=24),
    5: dict(kind="serve", V=20_000, s=1.0, max_len=20, req_median=20_000, req_sigma=1.0,
            req_min=1_000, req_max=1_000_000),
}


def single(n: int, V: int, s: float, max_len: int, seed: int) -> WordList:
    rng = np.random.Generator(np.random.PCG64(seed))
    vocab = make_vocabulary(rng, V, max_len, s)
    tok = draw_tokens(rng, vocab, n)
    chars, offsets = materialize(vocab, tok)
    return WordList(chars, offsets, None, dict(n=n, V=V, s=s, max_len=max_len, seed=seed))


def batch(n_docs: int, doc_min: int, doc_max: int, V: int, s: float, max_len: int,
          seed: int) -> WordList:
    """Documents of log-uniform size in [doc_min, doc_max] over one shared vocabulary."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vocab = make_vocabulary(rng, V, max_len, s)
    sizes = np.rint(np.exp(rng.uniform(np.log(doc_min), np.log(doc_max), size=n_docs)))
    sizes = sizes.astype(np.int64)
    toks = []
    for d in range(n_docs):
        r = np.random.Generator(np.random.PCG64(seed + DOC_SEED_STRIDE * (d + 1)))
        toks.append(draw_tokens(r, vocab, int(sizes[d])))
    tok = np.concatenate(toks) if toks else np.zeros(0, np.int64)
    chars, offsets = materialize(vocab, tok)
    doc_offsets = np.zeros(n_docs + 1, np.int64)
    np.cumsum(sizes, out=doc_offsets[1:])
    return WordList(chars, offsets, doc_offsets.astype(np.uint32),
                    dict(n_docs=n_docs, V=V, s=s, max_len=max_len, seed=seed))


def request_sizes(n_requests: int, median: float, sigma: float, lo: int, hi: int,
                  seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    x = np.rint(rng.lognormal(np.log(median), sigma, size=n_requests))
    return np.clip(x, lo, hi).astype(np.int64)


def config(cfg: int, scale: float = 1.0) -> WordList:
    """The seeded workload for a numbered config; ``scale`` shrinks sizes for tests."""
    c = CONFIGS[cfg]
    seed = SEED_BASE + cfg
    if c["kind"] == "single":
        n = max(1, int(round(c["n"] * scale)))
        wl = single(n, c["V"], c["s"], c["max_len"], seed)
        if "chunk" in c:
            wl.meta["chunk"] = c["chunk"]
        return wl
    if c["kind"] == "batch":
        nd = max(1, int(round(c["n_docs"] * scale)))
        return batch(nd, c["doc_min"], c["doc_max"], c["V"], c["s"], c["max_len"], seed)
    raise ValueError("config %d is a serving workload; use serving_requests()" % cfg)


def serving_requests(n_requests: int, scale: float = 1.0, cfg: int = 5):
    """Yield (size, WordList) per request: the request-size law over the config-2 vocabulary."""
    c = CONFIGS[cfg]
    seed = SEED_BASE + cfg
    rng = np.random.Generator(np.random.PCG64(seed))
    vocab = make_vocabulary(rng, c["V"], c["max_len"], c["s"])
    sizes = request_sizes(n_requests, c["req_median"] * scale, c["req_sigma"],
                          max(1, int(c["req_min"] * scale)), max(1, int(c["req_max"] * scale)),
                          seed)
    for r in range(n_requests):
        rr = np.random.Generator(np.random.PCG64(seed + REQUEST_SEED_STRIDE * (r + 1)))
        tok = draw_tokens(rr, vocab, int(sizes[r]))
        chars, offsets = materialize(vocab, tok)
        yield WordList(chars, offsets, None, dict(request=r, n=int(sizes[r])))


def from_words(words) -> WordList:
    """CSR word list from a sequence of bytes/str (tests and small examples)."""
    bs = [w.encode() if isinstance(w, str) else bytes(w) for w in words]
    offsets = np.zeros(len(bs) + 1, np.int64)
    np.cumsum([len(b) for b in bs], out=offsets[1:])
    chars = np.frombuffer(b"".join(bs), np.uint8).copy()
    return WordList(chars, offsets.astype(np.uint32))


def concat_docs(lists) -> WordList:
    """Several word lists as one batch (each list becomes one document)."""
    lists = list(lists)
    chars = np.concatenate([w.chars for w in lists]) if lists else np.zeros(0, np.uint8)
    offs = [np.zeros(1, np.int64)]
    base_c = 0
    doc = [0]
    for w in lists:
        offs.append(w.offsets[1:].astype(np.int64) - int(w.offsets[0]) + base_c)
        base_c += int(w.offsets[-1]) - int(w.offsets[0])
        doc.append(doc[-1] + w.n)
    offsets = np.concatenate(offs)
    return WordList(chars, offsets.astype(np.uint32), np.asarray(doc, np.uint32))


# Raw text for the tokenizer: a word list written out as prose.  Only bytes
# that carry no letters are added (spaces, line breaks, punctuation, digits in
# place of some separators), and some first letters are made capitals, so
# tokenizing with lower-case folding gives the word list back.
_PUNCT = np.frombuffer(b",.;:!?\")", np.uint8)
_OPEN = np.frombuffer(b"(\"", np.uint8)


def render_text(wl: WordList, seed: int) -> np.ndarray:
    """The whole word list as text (in pieces of _CHUNK words, each seeded on its own)."""
    parts = []
    for j, lo in enumerate(range(0, max(wl.n, 1), _CHUNK)):
        hi = min(wl.n, lo + _CHUNK)
        offs = wl.offsets[lo:hi + 1]
        parts.append(_render(wl.chars, offs, seed + j))
    return np.concatenate(parts) if len(parts) > 1 else parts[0]


def _render(chars: np.ndarray, offsets: np.ndarray, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = offsets.shape[0] - 1
    offs = offsets.astype(np.int64)
    L = np.diff(offs)
    pre = (rng.random(n) < 0.02).astype(np.int64)           # opening bracket or quote
    suf = (rng.random(n) < 0.15).astype(np.int64)           # trailing punctuation
    sep_kind = rng.random(n)
    sep = np.where(sep_kind < 0.02, 2, 1).astype(np.int64)  # some separators are a space and a digit
    size = pre + L + suf + sep
    start = np.zeros(n + 1, np.int64)
    np.cumsum(size, out=start[1:])
    out = np.full(int(start[-1]), ord(" "), np.uint8)
    if n == 0:
        return out
    # letters, with some first letters made capitals
    first = start[:-1] + pre
    dst = np.repeat(first - offs[:-1], L) + np.arange(int(offs[-1] - offs[0]), dtype=np.int64) + offs[0]
    out[dst] = chars[offs[0]:offs[-1]]
    cap = (rng.random(n) < 0.1) & (L > 0)
    out[first[cap]] -= 32
    out[start[:-1][pre == 1]] = _OPEN[rng.integers(0, _OPEN.size, int(pre.sum()))]
    after = first + L
    out[after[suf == 1]] = _PUNCT[rng.integers(0, _PUNCT.size, int(suf.sum()))]
    # separators: mostly a space, sometimes a line break, sometimes a space
    # followed by a digit (dropped from the run it starts)
    sp = after + suf
    line = sep_kind > 0.93
    out[sp[line]] = ord("\n")
    two = sep == 2
    out[sp[two] + 1] = ord("0") + rng.integers(0, 10, int(two.sum())).astype(np.uint8)
    return out
