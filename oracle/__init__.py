"""CPU oracle for the length-bucketed word sort -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  The GPU library never calls it and shares no
code with it.

Functions (host numpy arrays in, numpy arrays out):

* ``oracle_bubble``  -- the paper's sequential method: length lists (phase 2
  of "Pre-processing", section 3), bubble sort of each list (section 2,
  phase 3), lists concatenated shorter-first.  Plain C, ``oracle.c``.
* ``oracle_chunked`` -- the paper's parallel form (sections 3.2 and 4): chunks
  bubble-sorted alone, then merged.  Plain C.
* ``oracle_chunks``  -- the chunk step alone (section 4, each slave's bubble
  sort of its chunk): chunks sorted, not merged.  Plain C.
* ``oracle_def``     -- the definition the method reaches: indices ordered by
  the total order (length, bytes unsigned, index).  Plain C over qsort.
* ``oracle_sorted``  -- the same definition with Python's ``sorted``.
* ``oracle_def_parallel`` -- oracle_def on each length list, lists on host
  threads (for the CPU baseline on all cores).
* ``oracle_rank``    -- rank of one word under that order (O(n), for sampling
  outputs of inputs too large to sort on the CPU).
* ``paper_chunk_size`` -- chunk size = array size / number of processors
  (section 5, Results), rounded up so that the chunks cover the array.
* ``oracle_tokenize`` -- the first pre-processing phase (section 3): raw text
  to the word list, special characters removed.  Plain C.
* ``oracle_materialize`` -- the sorted words written out as text (section 4:
  the merged chunks are printed).  Plain C; ``oracle_materialize_batch`` runs
  it per document.

Parity: pinned by brute force over all permutations of tiny inputs, by
invariants, closed forms and Python's stable ``sorted`` (tests/test_oracle.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_LEN = 32
N_OFFSETS = MAX_LEN + 2

OK, INVALID_ARG, WORD_TOO_LONG, CAPACITY, OOM = 0, -1, -2, -3, -4
TOK_LOWER = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        for name in ("oracle_bubble", "oracle_def"):
            f = getattr(lib, name)
            f.argtypes = [u8p, u32p, ctypes.c_uint32, u32p, u32p]
            f.restype = ctypes.c_int
        for name in ("oracle_chunked", "oracle_chunks"):
            f = getattr(lib, name)
            f.argtypes = [u8p, u32p, ctypes.c_uint32, ctypes.c_uint32, u32p, u32p]
            f.restype = ctypes.c_int
        lib.oracle_rank.argtypes = [u8p, u32p, ctypes.c_uint32, ctypes.c_uint32]
        lib.oracle_rank.restype = ctypes.c_uint64
        lib.oracle_length_counts.argtypes = [u32p, ctypes.c_uint32, u64p]
        lib.oracle_length_counts.restype = ctypes.c_int
        lib.oracle_tokenize.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, u8p, u32p,
                                        ctypes.c_uint32, u32p]
        lib.oracle_tokenize.restype = ctypes.c_int
        lib.oracle_materialize.argtypes = [u8p, u32p, ctypes.c_uint32, u32p, ctypes.c_int, u8p]
        lib.oracle_materialize.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _prep(chars, offsets):
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    if chars.size == 0:
        chars = np.zeros(1, np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    return chars, offsets


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle returned %d" % code)
        self.code = code


def _call5(fn, chars, offsets, raise_on_error):
    chars, offsets = _prep(chars, offsets)
    n = offsets.shape[0] - 1
    perm = np.zeros(max(n, 1), np.uint32)
    boff = np.zeros(N_OFFSETS, np.uint32)
    rc = fn(_p(chars, ctypes.c_uint8), _p(offsets, ctypes.c_uint32), n,
            _p(perm, ctypes.c_uint32), _p(boff, ctypes.c_uint32))
    if rc != OK:
        if raise_on_error:
            raise OracleError(rc)
        return rc, None, None
    return rc, perm[:n], boff


def oracle_bubble(chars, offsets):
    """(perm, bucket_offsets) by per-length bubble sort."""
    _, perm, boff = _call5(_load().oracle_bubble, chars, offsets, True)
    return perm, boff


def oracle_def(chars, offsets):
    """(perm, bucket_offsets) by the total order (length, bytes, index)."""
    _, perm, boff = _call5(_load().oracle_def, chars, offsets, True)
    return perm, boff


def oracle_status(chars, offsets, fn: str = "oracle_bubble") -> int:
    """Return code of an oracle entry point (0 or a negative error)."""
    rc, _, _ = _call5(getattr(_load(), fn), chars, offsets, False)
    return rc


def _call_chunk(fn, chars, offsets, chunk):
    chars, offsets = _prep(chars, offsets)
    n = offsets.shape[0] - 1
    perm = np.zeros(max(n, 1), np.uint32)
    boff = np.zeros(N_OFFSETS, np.uint32)
    rc = fn(_p(chars, ctypes.c_uint8), _p(offsets, ctypes.c_uint32), n,
            int(chunk), _p(perm, ctypes.c_uint32), _p(boff, ctypes.c_uint32))
    if rc != OK:
        raise OracleError(rc)
    return perm[:n], boff


def oracle_chunked(chars, offsets, chunk: int):
    """(perm, bucket_offsets): chunks of each length list bubble-sorted alone, then merged."""
    return _call_chunk(_load().oracle_chunked, chars, offsets, chunk)


def oracle_chunks(chars, offsets, chunk: int):
    """(perm, bucket_offsets) after the chunk step alone: each length list's chunks of
    `chunk` words bubble-sorted, laid out one after another, NOT merged (section 4's
    slaves before the master's merge)."""
    return _call_chunk(_load().oracle_chunks, chars, offsets, chunk)


def oracle_rank(chars, offsets, i: int) -> int:
    chars, offsets = _prep(chars, offsets)
    n = offsets.shape[0] - 1
    return int(_load().oracle_rank(_p(chars, ctypes.c_uint8), _p(offsets, ctypes.c_uint32),
                                   n, int(i)))


def oracle_length_counts(offsets) -> np.ndarray:
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    out = np.zeros(MAX_LEN + 1, np.uint64)
    rc = _load().oracle_length_counts(_p(offsets, ctypes.c_uint32), offsets.shape[0] - 1,
                                      _p(out, ctypes.c_uint64))
    if rc != OK:
        raise OracleError(rc)
    return out


def oracle_sorted(words):
    """Python twin of the definition: ``sorted`` is stable, so equal words keep index order."""
    ws = [w.encode() if isinstance(w, str) else bytes(w) for w in words]
    perm = sorted(range(len(ws)), key=lambda i: (len(ws[i]), ws[i]))
    boff = [0] * N_OFFSETS
    for w in ws:
        boff[len(w) + 1] += 1
    for L in range(1, N_OFFSETS):
        boff[L] += boff[L - 1]
    return np.asarray(perm, np.uint32), np.asarray(boff, np.uint32)


def oracle_batch(chars, offsets, doc_offsets, fn: str = "oracle_bubble", threads: int = 0):
    """Each document sorted on its own (doc-local indices); documents run on host threads.

    Returns (perm [N], bucket_offsets [n_docs, 34])."""
    chars, offsets = _prep(chars, offsets)
    doc_offsets = np.asarray(doc_offsets, dtype=np.int64)
    nd = doc_offsets.shape[0] - 1
    N = int(doc_offsets[-1]) if nd >= 0 else 0
    perm = np.zeros(max(N, 1), np.uint32)
    boff = np.zeros((max(nd, 1), N_OFFSETS), np.uint32)
    f = getattr(_load(), fn)

    def one(d):
        lo, hi = int(doc_offsets[d]), int(doc_offsets[d + 1])
        sub_off = np.ascontiguousarray(offsets[lo:hi + 1])
        p = np.zeros(max(hi - lo, 1), np.uint32)
        b = np.zeros(N_OFFSETS, np.uint32)
        rc = f(_p(chars, ctypes.c_uint8), _p(sub_off, ctypes.c_uint32), hi - lo,
               _p(p, ctypes.c_uint32), _p(b, ctypes.c_uint32))
        if rc != OK:
            raise OracleError(rc)
        perm[lo:hi] = p[:hi - lo]
        boff[d] = b

    threads = threads or len(os.sched_getaffinity(0))
    # largest documents first so the pool stays busy
    order = sorted(range(nd), key=lambda d: -(int(doc_offsets[d + 1]) - int(doc_offsets[d])))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, order))
    return perm[:N], boff[:nd]


def oracle_def_parallel(chars, offsets, threads: int = 0):
    """oracle_def with the length lists on host threads: the words are put
    into one list per length (phase 2 of section 3), each list is sorted by
    oracle_def on a thread of its own, and the lists are laid out shorter
    first.  Returns (perm, bucket_offsets) equal to oracle_def's."""
    chars, offsets = _prep(chars, offsets)
    n = offsets.shape[0] - 1
    offs = offsets.astype(np.int64)
    lens = offs[1:] - offs[:-1]
    if n and (lens.min() < 0 or lens.max() > MAX_LEN):
        raise OracleError(INVALID_ARG if lens.min() < 0 else WORD_TOO_LONG)
    order = np.argsort(lens, kind="stable")             # indices of each length, in input order
    counts = np.bincount(lens, minlength=MAX_LEN + 1)[:MAX_LEN + 1] if n else np.zeros(MAX_LEN + 1, np.int64)
    boff = np.zeros(N_OFFSETS, np.uint32)
    boff[1:] = np.cumsum(counts)
    perm = np.zeros(max(n, 1), np.uint32)

    def one(L):
        lo, hi = int(boff[L]), int(boff[L + 1])
        if hi == lo:
            return
        idx = order[lo:hi]
        # the list's words back to back: list word k is chars[sub[k] .. sub[k] + L)
        starts = offs[idx]
        sub_chars = chars[(starts[:, None] + np.arange(L)[None, :]).reshape(-1)] if L else np.zeros(1, np.uint8)
        sub_offs = (np.arange(hi - lo + 1, dtype=np.int64) * L).astype(np.uint32)
        p, _ = oracle_def(sub_chars, sub_offs)
        perm[lo:hi] = idx[p.astype(np.int64)]

    threads = threads or len(os.sched_getaffinity(0))
    # longest lists first so the pool stays busy
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, sorted(range(MAX_LEN + 1), key=lambda L: -int(counts[L]))))
    return perm[:n], boff


def paper_chunk_size(array_size: int, processors: int) -> int:
    """Chunk size = array size / number of processors (section 5), rounded up."""
    if processors <= 0:
        raise ValueError("processors must be positive")
    return -(-int(array_size) // int(processors))


def oracle_tokenize(text, flags: int = 0, max_words=None):
    """(chars, offsets) of the words of raw text: runs between ASCII whitespace,
    letters only, other bytes removed (flags & TOK_LOWER: lower case)."""
    t = np.frombuffer(bytes(text), np.uint8) if not isinstance(text, np.ndarray) else \
        np.ascontiguousarray(text, dtype=np.uint8)
    n = t.shape[0]
    cap = (n + 1) // 2 if max_words is None else int(max_words)
    buf = t if n else np.zeros(1, np.uint8)
    chars = np.zeros(max(n, 1), np.uint8)
    offs = np.zeros(cap + 1, np.uint32)
    nw = np.zeros(1, np.uint32)
    rc = _load().oracle_tokenize(_p(buf, ctypes.c_uint8), n, int(flags), _p(chars, ctypes.c_uint8),
                                 _p(offs, ctypes.c_uint32), cap, _p(nw, ctypes.c_uint32))
    if rc != OK:
        raise OracleError(rc)
    k = int(nw[0])
    return chars[:int(offs[k])].copy(), offs[:k + 1].copy()


def oracle_materialize(chars, offsets, perm, sep: int = 10) -> bytes:
    """Word perm[k] for k = 0..n-1, each followed by byte ``sep`` (none if sep < 0)."""
    chars, offsets = _prep(chars, offsets)
    n = offsets.shape[0] - 1
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    if perm.shape[0] != n:
        raise OracleError(INVALID_ARG)
    size = int(offsets[-1]) - int(offsets[0]) + (n if sep >= 0 else 0) if n else 0
    out = np.zeros(max(size, 1), np.uint8)
    pp = perm if n else np.zeros(1, np.uint32)
    rc = _load().oracle_materialize(_p(chars, ctypes.c_uint8), _p(offsets, ctypes.c_uint32), n,
                                    _p(pp, ctypes.c_uint32), int(sep), _p(out, ctypes.c_uint8))
    if rc != OK:
        raise OracleError(rc)
    return out[:size].tobytes()


def oracle_materialize_batch(chars, offsets, doc_offsets, perm, sep: int = 10) -> bytes:
    """Per document (doc-local perm), documents back to back."""
    chars, offsets = _prep(chars, offsets)
    doc_offsets = np.asarray(doc_offsets, dtype=np.int64)
    perm = np.asarray(perm, dtype=np.uint32)
    parts = []
    for d in range(doc_offsets.shape[0] - 1):
        lo, hi = int(doc_offsets[d]), int(doc_offsets[d + 1])
        parts.append(oracle_materialize(chars, offsets[lo:hi + 1], perm[lo:hi], sep))
    return b"".join(parts)
