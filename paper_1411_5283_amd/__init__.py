"""MI355X-native length-bucketed word sort (arXiv:1411.5283's method on gfx950).

Thin ctypes binding over ``libsortwords.so`` (built from ``csrc/`` by
``build.py``).  Every step of the sort runs in the library's HIP kernels;
this module only marshals arguments.  Device buffers are torch CUDA tensors
(torch is used for device memory and streams only).  Word offsets and
permutations are uint32 on the device and travel as int32 tensors holding
the same bits.

The C entry points and their semantics are declared in
``include/sort_words.h``; the functions here carry the same names.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsortwords.so")

MAX_LEN = 32
NUM_OFFSETS = MAX_LEN + 2
NUM_CLASSES = 5           # key classes: lengths 0-4, 5-8, 9-16, 17-24, 25-32

OK, ERR_INVALID_ARG, ERR_WORD_TOO_LONG, ERR_WORKSPACE, ERR_OOM, ERR_HIP = 0, -1, -2, -3, -4, -5
_STATUS_NAMES = {0: "SW_OK", -1: "SW_ERR_INVALID_ARG", -2: "SW_ERR_WORD_TOO_LONG",
                 -3: "SW_ERR_WORKSPACE", -4: "SW_ERR_OOM", -5: "SW_ERR_HIP"}


class SortWordsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


FLAG_SERIAL_CLASSES = 1
FLAG_PACKED_FIRST = 2
FLAG_SCHEDULE_BESIDE_SCATTER = 4
FLAG_ORDER_SHIFT = 8        # bits 8..14: index (0..119) of the classes' enqueue order
FLAG_ORDER_MASK = 127 << FLAG_ORDER_SHIFT
NUM_ORDERS = 120


def class_order(index: int) -> list:
    """The classes' enqueue order that order index 0..119 names (the orders of
    0..4 in lexicographic order), for reporting a configuration."""
    import itertools
    return list(list(itertools.permutations(range(NUM_CLASSES)))[index])


class sw_config(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32 * NUM_CLASSES), ("variant", ctypes.c_uint32 * NUM_CLASSES),
                ("flags", ctypes.c_uint32), ("merge", ctypes.c_uint32 * NUM_CLASSES)]


class sw_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("max_batch_words", ctypes.c_uint32),
                ("max_batch_docs", ctypes.c_uint32), ("copy_threads", ctypes.c_uint32),
                ("max_batch_chars", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("min_batch_words", ctypes.c_uint32), ("max_wait_us", ctypes.c_uint32)]


class sw_server_counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("completed", "failed", "words", "batches", "bytes_in_use",
                                               "max_bytes_in_use")]


_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsortwords.so is not built; run __graft_entry__.build() or "
                           "python -m paper_1411_5283_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
    sig = {
        "sort_words": ([vp, vp, u32, vp, vp], i32),
        "sort_words_workspace_size": ([u32, u32], sz),
        "sort_words_ex": ([vp, vp, u32, vp, vp, vp, sz, vp], i32),
        "sort_words_batch": ([vp, vp, vp, u32, vp, vp, vp, sz, vp], i32),
        "sort_words_plain": ([vp, vp, vp, u32, vp, vp, vp, sz, vp], i32),
        "sort_words_unbucketed": ([vp, vp, u32, vp, vp, vp, sz, vp], i32),
        "sort_words_chunks": ([vp, vp, u32, u32, vp, vp, vp, sz, vp], i32),
        "sort_words_noalloc": ([vp, vp, u32, vp, vp, vp, vp], i32),
        "sort_words_status": ([vp, vp], i32),
        "sw_plan_create": ([u32, u32, ctypes.c_uint64, vp, ctypes.POINTER(vp)], i32),
        "sw_plan_run": ([vp, vp, vp, vp, u32, u32, vp, vp], i32),
        "sw_plan_run_text": ([vp, vp, vp, vp, u32, u32, vp, vp, i32, vp], i32),
        "sw_plan_status": ([vp], i32),
        "sw_plan_status_async": ([vp, vp], i32),
        "sort_words_status_async": ([vp, vp, vp], i32),
        "sort_words_decode_status": ([u32], i32),
        "sw_plan_destroy": ([vp], None),
        "sw_get_config": ([ctypes.POINTER(sw_config)], i32),
        "sw_set_config": ([ctypes.POINTER(sw_config)], i32),
        "sw_num_variants": ([i32], i32),
        "sw_num_merges": ([i32], i32),
        "sw_variant_tiles": ([i32, i32, ctypes.POINTER(u32), ctypes.POINTER(u32)], i32),
        "sw_profile_enable": ([i32], i32),
        "sw_profile_reset": ([], i32),
        "sw_profile_read": ([i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(u32),
                             ctypes.POINTER(ctypes.c_double)], i32),
        "sort_words_tokenize_workspace_size": ([ctypes.c_uint64], sz),
        "sort_words_tokenize": ([vp, ctypes.c_uint64, u32, vp, vp, u32, vp, vp, sz, vp], i32),
        "sort_words_materialize": ([vp, vp, vp, u32, u32, vp, vp, i32, vp, vp, vp], i32),
        "sw_server_create": ([ctypes.POINTER(sw_server_config), ctypes.POINTER(vp)], i32),
        "sw_server_submit": ([vp, vp, vp, u32, vp, vp, ctypes.POINTER(ctypes.c_uint64)], i32),
        "sw_server_wait": ([vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)], i32),
        "sw_server_stats": ([vp, ctypes.POINTER(sw_server_counts)], i32),
        "sw_server_fixed_bytes": ([ctypes.POINTER(sw_server_config)], sz),
        "sw_server_request_bytes": ([u32, ctypes.c_uint64], ctypes.c_uint64),
        "sw_server_destroy": ([vp], None),
        "sort_words_last_error": ([], ctypes.c_char_p),
        "sort_words_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


EXPORTED = ("sort_words", "sort_words_workspace_size", "sort_words_ex", "sort_words_batch",
            "sort_words_plain", "sort_words_unbucketed", "sort_words_chunks", "sort_words_noalloc",
            "sort_words_status", "sort_words_status_async",
            "sort_words_decode_status", "sw_plan_create", "sw_plan_run", "sw_plan_run_text",
            "sw_plan_status", "sw_plan_status_async", "sw_plan_destroy", "sw_get_config", "sw_set_config",
            "sw_num_variants", "sw_num_merges", "sw_variant_tiles", "sw_profile_enable", "sw_profile_reset",
            "sw_profile_read", "sort_words_tokenize_workspace_size", "sort_words_tokenize",
            "sort_words_materialize", "sw_server_create", "sw_server_submit", "sw_server_wait",
            "sw_server_stats", "sw_server_fixed_bytes", "sw_server_request_bytes", "sw_server_destroy",
            "sort_words_last_error",
            "sort_words_version")


def _check(rc: int) -> int:
    if rc != OK:
        raise SortWordsError(rc, lib().sort_words_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    p = t.data_ptr()
    return p or None


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


# ------------------------------------------------------------------ entry points
def sort_words(chars, offsets, n, out_perm, out_bucket_offsets) -> int:
    """Synchronous sort on the null stream (library-owned workspace)."""
    return _check(lib().sort_words(_ptr(chars), _ptr(offsets), int(n), _ptr(out_perm),
                                   _ptr(out_bucket_offsets)))


def sort_words_workspace_size(max_words: int, max_docs: int = 1) -> int:
    return int(lib().sort_words_workspace_size(int(max_words), int(max_docs)))


def sort_words_ex(chars, offsets, n, out_perm, out_bucket_offsets, workspace, stream=None) -> int:
    return _check(lib().sort_words_ex(_ptr(chars), _ptr(offsets), int(n), _ptr(out_perm),
                                      _ptr(out_bucket_offsets), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 32 << 20


def sort_words_noalloc(chars, offsets, n, out_perm, out_bucket_offsets, out_status, stream=None) -> int:
    """sort_words_ex on the library's fixed scratch (no allocation; asynchronous).
    out_status: a 1-element int32 device tensor that receives the device status word."""
    return _check(lib().sort_words_noalloc(_ptr(chars), _ptr(offsets), int(n), _ptr(out_perm),
                                           _ptr(out_bucket_offsets), _ptr(out_status), _stream(stream)))


def sort_words_batch(chars, offsets, doc_offsets, n_docs, out_perm, out_bucket_offsets, workspace,
                     stream=None) -> int:
    return _check(lib().sort_words_batch(_ptr(chars), _ptr(offsets), _ptr(doc_offsets), int(n_docs),
                                         _ptr(out_perm), _ptr(out_bucket_offsets), _ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream)))


def sort_words_plain(chars, offsets, doc_offsets, n_docs, out_perm, out_bucket_offsets, workspace,
                     stream=None) -> int:
    return _check(lib().sort_words_plain(_ptr(chars), _ptr(offsets), _ptr(doc_offsets), int(n_docs),
                                         _ptr(out_perm), _ptr(out_bucket_offsets), _ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream)))


def sort_words_unbucketed(chars, offsets, n, out_perm, out_bucket_offsets, workspace, stream=None) -> int:
    """The baseline without length lists (asynchronous; errors via sort_words_status)."""
    return _check(lib().sort_words_unbucketed(_ptr(chars), _ptr(offsets), int(n), _ptr(out_perm),
                                              _ptr(out_bucket_offsets), _ptr(workspace),
                                              workspace.numel() * workspace.element_size(), _stream(stream)))


def sort_words_chunks(chars, offsets, n, chunk, out_perm, out_bucket_offsets, workspace, stream=None) -> int:
    """The chunk step alone: each length list's chunks of `chunk` words sorted, not merged (synchronous)."""
    return _check(lib().sort_words_chunks(_ptr(chars), _ptr(offsets), int(n), int(chunk), _ptr(out_perm),
                                          _ptr(out_bucket_offsets), _ptr(workspace),
                                          workspace.numel() * workspace.element_size(), _stream(stream)))


def sort_words_status(workspace, stream=None) -> int:
    """Device status of the last call enqueued with this workspace (raises on error)."""
    return _check(lib().sort_words_status(_ptr(workspace), _stream(stream)))


def sort_words_status_code(workspace, stream=None) -> int:
    return int(lib().sort_words_status(_ptr(workspace), _stream(stream)))


def sort_words_status_async(workspace, status_dst, stream=None) -> int:
    """Enqueue a copy of the device status word into status_dst (a 1-element int32 tensor)."""
    return _check(lib().sort_words_status_async(_ptr(workspace), _ptr(status_dst), _stream(stream)))


def decode_status(word: int) -> int:
    return int(lib().sort_words_decode_status(int(word) & 0xFFFFFFFF))


class Plan:
    """Graph-captured persistent plan (sw_plan_*)."""

    def __init__(self, max_words: int, max_docs: int = 1, stream=None, max_chars: int = (1 << 32) - 1):
        h = ctypes.c_void_p()
        s = None if stream is None else _stream(stream)
        _check(lib().sw_plan_create(int(max_words), int(max_docs), int(max_chars), s, ctypes.byref(h)))
        self._h = h
        self.max_words, self.max_docs, self.max_chars = int(max_words), int(max_docs), int(max_chars)

    def run(self, chars, offsets, doc_offsets, n_docs, n_words, out_perm, out_bucket_offsets) -> int:
        return _check(lib().sw_plan_run(self._h, _ptr(chars), _ptr(offsets), _ptr(doc_offsets),
                                        int(n_docs), int(n_words), _ptr(out_perm),
                                        _ptr(out_bucket_offsets)))

    def run_text(self, chars, offsets, doc_offsets, n_docs, n_words, out_perm, out_bucket_offsets, sep,
                 out_text) -> int:
        """run() plus the sorted text written from the sorted keys (sw_plan_run_text);
        out_text: text_size(...) bytes, the layout materialize() writes."""
        return _check(lib().sw_plan_run_text(self._h, _ptr(chars), _ptr(offsets), _ptr(doc_offsets),
                                             int(n_docs), int(n_words), _ptr(out_perm),
                                             _ptr(out_bucket_offsets), int(sep), _ptr(out_text)))

    def status(self) -> int:
        return _check(lib().sw_plan_status(self._h))

    def status_code(self) -> int:
        return int(lib().sw_plan_status(self._h))

    def status_async(self, status_dst) -> int:
        """Enqueue a copy of the device status word into status_dst (1-element int32 tensor)."""
        return _check(lib().sw_plan_status_async(self._h, _ptr(status_dst)))

    def close(self):
        if self._h:
            lib().sw_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def get_config() -> dict:
    c = sw_config()
    _check(lib().sw_get_config(ctypes.byref(c)))
    return {"chunk": list(c.chunk), "variant": list(c.variant), "flags": int(c.flags), "merge": list(c.merge)}


def set_config(chunk=None, variant=None, flags=None, merge=None) -> dict:
    cur = get_config()
    for name, v in (("chunk", chunk), ("variant", variant), ("merge", merge)):
        if v is not None and len(v) != NUM_CLASSES:
            raise ValueError("%s: one value per key class (%d), got %d" % (name, NUM_CLASSES, len(v)))
    c = sw_config()
    for k in range(NUM_CLASSES):
        c.chunk[k] = int((chunk if chunk is not None else cur["chunk"])[k])
        c.variant[k] = int((variant if variant is not None else cur["variant"])[k])
        c.merge[k] = int((merge if merge is not None else cur["merge"])[k])
    c.flags = int(flags if flags is not None else cur["flags"])
    _check(lib().sw_set_config(ctypes.byref(c)))
    return get_config()


def num_variants(cls: int) -> int:
    return int(lib().sw_num_variants(int(cls)))


def num_merges(cls: int) -> int:
    """Choices of sw_config.merge[cls]: 0 two-way levels, 1.. four-way configurations."""
    return int(lib().sw_num_merges(int(cls)))


def variant_tiles(cls: int, variant: int) -> tuple[int, int]:
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().sw_variant_tiles(int(cls), int(variant), ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def profile_enable(on: bool = True):
    _check(lib().sw_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().sw_profile_reset())


def profile_read() -> dict:
    """{kernel family: (launches, milliseconds)} since the last reset."""
    n = 64
    names = (ctypes.c_char_p * n)()
    launches = (ctypes.c_uint32 * n)()
    ms = (ctypes.c_double * n)()
    k = lib().sw_profile_read(n, names, launches, ms)
    if k < 0:
        _check(k)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(k)}


def version() -> str:
    return lib().sort_words_version().decode()


# ------------------------------------------------------------------ around the sort
TOK_LOWER = 1


def tokenize_workspace_size(n_bytes: int) -> int:
    return int(lib().sort_words_tokenize_workspace_size(int(n_bytes)))


def tokenize(text, n_bytes, flags, out_chars, out_offsets, max_words, out_n_words, workspace, stream=None):
    """sort_words_tokenize on device tensors (asynchronous; errors via sort_words_status(workspace))."""
    return _check(lib().sort_words_tokenize(_ptr(text), int(n_bytes), int(flags), _ptr(out_chars),
                                            _ptr(out_offsets), int(max_words), _ptr(out_n_words),
                                            _ptr(workspace), workspace.numel(), _stream(stream)))


def materialize(chars, offsets, doc_offsets, n_docs, n_words, perm, bucket_offsets, sep, out_text,
                out_status, stream=None):
    """sort_words_materialize on device tensors (asynchronous; out_status nonzero = a check failed)."""
    return _check(lib().sort_words_materialize(_ptr(chars), _ptr(offsets), _ptr(doc_offsets), int(n_docs),
                                               int(n_words), _ptr(perm), _ptr(bucket_offsets), int(sep),
                                               _ptr(out_text), _ptr(out_status), _stream(stream)))


def text_size(wl, sep: int) -> int:
    """Bytes of the sorted text of a word list (one separator per word when sep >= 0)."""
    n = wl.n
    return int(wl.offsets[n]) - int(wl.offsets[0]) + (n if sep >= 0 else 0) if n else 0


# ------------------------------------------------------------------ serving (native loop)
class NativeServer:
    """The library's serving loop (sw_server_*): requests are host arrays;
    results come back as host arrays.  A request's arrays are kept alive here
    until it has been waited for."""

    def __init__(self, slots: int = 2, max_batch_words: int = 1 << 22, max_batch_docs: int = 256,
                 max_batch_chars: int | None = None, budget_bytes: int = 8 << 30, min_batch_words: int = 0,
                 max_wait_us: int = 0, copy_threads: int = 4):
        self.cfg = sw_server_config(int(slots), int(max_batch_words), int(max_batch_docs), int(copy_threads),
                                    int(max_batch_chars or max_batch_words * 8), int(budget_bytes),
                                    int(min_batch_words), int(max_wait_us))
        h = ctypes.c_void_p()
        _check(lib().sw_server_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self._live = {}

    def fixed_bytes(self) -> int:
        return int(lib().sw_server_fixed_bytes(ctypes.byref(self.cfg)))

    @staticmethod
    def request_bytes(n_words: int, n_chars: int) -> int:
        """Bytes of the budget a request holds from admission until its batch completes."""
        return int(lib().sw_server_request_bytes(int(n_words), int(n_chars)))

    def submit(self, chars, offsets) -> int:
        """Queue one request; returns its ticket (raises at once if it is refused)."""
        chars = np.ascontiguousarray(chars, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
        n = offsets.shape[0] - 1
        if n < 0:
            raise SortWordsError(ERR_INVALID_ARG, "offsets must hold n+1 entries")
        perm = np.empty(max(n, 1), np.uint32)
        boff = np.empty(NUM_OFFSETS, np.uint32)
        t = ctypes.c_uint64()
        cp = chars.ctypes.data if chars.size else None
        _check(lib().sw_server_submit(self._h, cp, offsets.ctypes.data, n, perm.ctypes.data,
                                      boff.ctypes.data, ctypes.byref(t)))
        self._live[t.value] = (chars, offsets, perm, boff, n)
        return t.value

    def wait(self, ticket: int):
        """(perm, bucket_offsets, latency_s) of a request; raises if its batch failed."""
        lat = ctypes.c_double()
        rc = lib().sw_server_wait(self._h, int(ticket), ctypes.byref(lat))
        chars, offsets, perm, boff, n = self._live.pop(int(ticket))
        _check(rc)
        return perm[:n], boff, float(lat.value)

    def stats(self) -> dict:
        c = sw_server_counts()
        _check(lib().sw_server_stats(self._h, ctypes.byref(c)))
        return {k: int(getattr(c, k)) for k, _ in c._fields_}

    def close(self):
        if self._h:
            lib().sw_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ host helpers
def device_words(wl, device="cuda"):
    """Copy a wordgen.WordList to the device: (chars u8, offsets i32[n+1], doc_offsets or None)."""
    import torch
    chars = torch.from_numpy(np.ascontiguousarray(wl.chars)).to(device)
    offsets = torch.from_numpy(np.ascontiguousarray(wl.offsets, dtype=np.uint32).view(np.int32)).to(device)
    docs = None
    if wl.doc_offsets is not None:
        docs = torch.from_numpy(np.ascontiguousarray(wl.doc_offsets, dtype=np.uint32).view(np.int32)).to(device)
    return chars, offsets, docs


def to_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def sort_wordlist(wl, device="cuda"):
    """Sort a host word list on the GPU (single document: sort_words; batch: sort_words_batch).

    Returns numpy (perm uint32[n], bucket_offsets uint32[34] or [n_docs, 34])."""
    import torch
    chars, offsets, docs = device_words(wl, device)
    n = wl.n
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    if docs is None:
        boff = torch.empty(NUM_OFFSETS, dtype=torch.int32, device=device)
        sort_words(chars, offsets, n, perm, boff)
        return to_u32(perm)[:n], to_u32(boff)
    nd = wl.n_docs
    boff = torch.empty(max(nd, 1) * NUM_OFFSETS, dtype=torch.int32, device=device)
    ws = torch.empty(sort_words_workspace_size(n, nd), dtype=torch.uint8, device=device)
    sort_words_batch(chars, offsets, docs, nd, perm, boff, ws)
    sort_words_status(ws)
    return to_u32(perm)[:n], to_u32(boff)[:nd * NUM_OFFSETS].reshape(nd, NUM_OFFSETS)


# ------------------------------------------------------------------ conveniences
def sort_strings(words, device="cuda"):
    """Sort a list of words (str or bytes, at most MAX_LEN bytes each) on the
    GPU by (length, bytes unsigned, position); returns (the sorted list,
    the permutation as uint32)."""
    from . import wordgen
    words = list(words)
    perm, _ = sort_wordlist(wordgen.from_words(words), device)
    return [words[i] for i in perm], perm


def sort_text(text, lower: bool = False, sep: int = 10, device="cuda") -> bytes:
    """Raw text in, sorted words out, every step on the GPU: the words are the
    runs between ASCII whitespace with their letters kept (sort_words_tokenize,
    lower case on request), sorted by (length, bytes, position) (sort_words),
    and written each followed by byte `sep`, or back to back when sep < 0
    (sort_words_materialize)."""
    import torch
    raw = np.frombuffer(bytes(text), np.uint8)
    nb = int(raw.size)
    t = torch.from_numpy(raw.copy() if nb else np.zeros(1, np.uint8)).to(device)
    max_words = (nb + 1) // 2
    chars = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    offs = torch.empty(max_words + 1, dtype=torch.int32, device=device)
    nw = torch.zeros(1, dtype=torch.int32, device=device)
    ws = torch.empty(tokenize_workspace_size(nb), dtype=torch.uint8, device=device)
    tokenize(t, nb, TOK_LOWER if lower else 0, chars, offs, max_words, nw, ws)
    sort_words_status(ws)
    n = int(nw.cpu()[0])
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    boff = torch.empty(NUM_OFFSETS, dtype=torch.int32, device=device)
    sort_words(chars, offs, n, perm, boff)
    size = int(offs[n].item()) + (n if sep >= 0 else 0) if n else 0
    out = torch.empty(max(size, 1), dtype=torch.uint8, device=device)
    st = torch.zeros(1, dtype=torch.int32, device=device)
    materialize(chars, offs, None, 1, n, perm, boff, sep, out, st)
    torch.cuda.synchronize()
    if int(st.cpu()[0]):
        raise SortWordsError(ERR_INVALID_ARG, "sort_text: the text writer's checks failed")
    return out[:size].cpu().numpy().tobytes()
