"""The C ABI library: it loads without a GPU and exports every declared symbol."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sort_words.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sort_words", "sort_words_ex", "sort_words_batch", "sort_words_plain",
                 "sort_words_status", "sort_words_workspace_size", "sw_plan_create", "sw_plan_run",
                 "sw_plan_destroy", "sort_words_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1411_5283_amd as sw
    if not os.path.exists(sw.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(sw.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(sw.EXPORTED) == set(declared_functions())


def test_host_side_calls_without_gpu():
    import paper_1411_5283_amd as sw
    if not os.path.exists(sw.LIB_PATH):
        pytest.skip("library not built")
    L = sw.lib()
    assert sw.version().startswith("sortwords-gfx950")
    # workspace sizes: monotone in words and documents; 0 when out of range
    a = sw.sort_words_workspace_size(1000, 1)
    b = sw.sort_words_workspace_size(100000, 1)
    c = sw.sort_words_workspace_size(100000, 4096)
    assert 0 < a < b < c
    assert sw.sort_words_workspace_size(1000, 0xFFFFFFFF) == 0
    # at most 2^32 - 2 words (every index below the chunk sort's fill key)
    assert sw.sort_words_workspace_size(0xFFFFFFFF, 1) == 0
    # argument validation happens on the host before any device call
    assert L.sort_words(None, None, 5, None, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_ex(None, None, 0, None, None, None, 0, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_batch(None, None, None, 1, None, None, None, 0, None) == sw.ERR_INVALID_ARG
    assert b"null" in L.sort_words_last_error()
    # the chunk step checks its chunk size, the no-allocation form its
    # arguments and its capacity, before any device call
    dummy = ctypes.create_string_buffer(64)
    p = ctypes.addressof(dummy)
    assert L.sort_words_chunks(p, p, 3, 3, p, p, p, 1 << 20, None) == sw.ERR_INVALID_ARG
    assert b"power of two" in L.sort_words_last_error()
    assert L.sort_words_chunks(p, p, 3, 2048, p, p, p, 1 << 20, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_noalloc(p, p, 3, p, p, None, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_noalloc(p, p, 1 << 22, p, p, p, None) == sw.ERR_WORKSPACE
    assert b"scratch" in L.sort_words_last_error()
    # config validation
    cfg = sw.sw_config()
    assert L.sw_get_config(ctypes.byref(cfg)) == 0
    bad = sw.sw_config()
    for k in range(sw.NUM_CLASSES):
        bad.chunk[k] = 48            # not a power of two
    assert L.sw_set_config(ctypes.byref(bad)) == sw.ERR_INVALID_ARG
    flagged = sw.sw_config()
    ctypes.memmove(ctypes.byref(flagged), ctypes.byref(cfg), ctypes.sizeof(cfg))
    flagged.flags = 8                # no such flag
    assert L.sw_set_config(ctypes.byref(flagged)) == sw.ERR_INVALID_ARG
    flagged.flags = sw.FLAG_SERIAL_CLASSES | sw.FLAG_PACKED_FIRST | sw.FLAG_SCHEDULE_BESIDE_SCATTER
    assert L.sw_set_config(ctypes.byref(flagged)) == 0
    assert sw.get_config()["flags"] == 7
    flagged.flags = 120 << sw.FLAG_ORDER_SHIFT    # only 120 class orders
    assert L.sw_set_config(ctypes.byref(flagged)) == sw.ERR_INVALID_ARG
    flagged.flags = 119 << sw.FLAG_ORDER_SHIFT
    assert L.sw_set_config(ctypes.byref(flagged)) == 0
    assert sw.class_order(0) == [0, 1, 2, 3, 4] and sw.class_order(1) == [0, 1, 2, 4, 3]
    assert sw.class_order(119) == [4, 3, 2, 1, 0]
    with pytest.raises(ValueError):
        sw.set_config(chunk=[16] * 4)              # one value per class
    assert L.sw_set_config(ctypes.byref(cfg)) == 0
    assert sw.num_variants(0) >= 1 and sw.num_variants(7) == 0
    t, p = sw.variant_tiles(0, 0)
    assert t >= 1024 and p >= 1024 and (t & (t - 1)) == 0


def test_text_entry_points_validate_on_host():
    """Argument errors of the tokenizer and the text writer are found before any GPU call."""
    import paper_1411_5283_amd as sw
    L = sw.lib()
    assert L.sort_words_tokenize_workspace_size(1 << 32) == 0
    assert L.sort_words_tokenize_workspace_size(0) > 0
    # null outputs, a text of 2^32 bytes, unknown flags
    assert L.sort_words_tokenize(None, 10, 0, None, None, 4, None, None, 0, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_tokenize(1, 1 << 32, 0, 1, 1, 4, 1, 1, 1 << 20, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_tokenize(1, 10, 6, 1, 1, 4, 1, 1, 1 << 20, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_tokenize(1, 10, 0, 1, 1, 4, 1, 1, 8, None) == sw.ERR_WORKSPACE
    # the text writer: null pointers, a separator above 255, n_docs without doc_offsets
    assert L.sort_words_materialize(None, None, None, 1, 0, None, None, 10, None, None, None) == sw.ERR_INVALID_ARG
    # sort + text: a null plan
    assert L.sw_plan_run_text(None, None, None, None, 1, 0, None, None, 10, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_materialize(16, 16, None, 1, 5, 16, 16, 256, 16, 16, None) == sw.ERR_INVALID_ARG
    assert b"separator" in L.sort_words_last_error()
    assert L.sort_words_materialize(16, 16, None, 2, 5, 16, 16, 10, 16, 16, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_materialize(16, 16, 16, 0, 5, 16, 16, 10, 16, 16, None) == sw.ERR_INVALID_ARG


def test_unbucketed_validates_on_host():
    import paper_1411_5283_amd as sw
    L = sw.lib()
    assert L.sort_words_unbucketed(None, None, 0, None, None, None, 0, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_unbucketed(1, 1, 5, None, 1, 1, 1 << 20, None) == sw.ERR_INVALID_ARG
    assert L.sort_words_unbucketed(16, 16, 5, 16, 16, 16, 16, None) == sw.ERR_WORKSPACE


def test_server_validates_on_host():
    import ctypes
    import paper_1411_5283_amd as sw
    L = sw.lib()
    h = ctypes.c_void_p()
    bad = [sw.sw_server_config(0, 1000, 8, 0, 1 << 20, 1 << 30, 0, 0),        # no slot
           sw.sw_server_config(9, 1000, 8, 0, 1 << 20, 1 << 30, 0, 0),        # too many slots
           sw.sw_server_config(2, 0, 8, 0, 1 << 20, 1 << 30, 0, 0),           # empty batches
           sw.sw_server_config(2, 1000, 8, 65, 1 << 20, 1 << 30, 0, 0),       # too many copy threads
           sw.sw_server_config(2, 1000, 8, 0, 1 << 32, 1 << 30, 0, 0)]        # 2^32 characters
    for cfg in bad:
        assert L.sw_server_create(ctypes.byref(cfg), ctypes.byref(h)) == sw.ERR_INVALID_ARG
    assert L.sw_server_create(None, ctypes.byref(h)) == sw.ERR_INVALID_ARG
    t = ctypes.c_uint64()
    assert L.sw_server_submit(None, None, None, 0, None, None, ctypes.byref(t)) == sw.ERR_INVALID_ARG
    assert L.sw_server_wait(None, 1, None) == sw.ERR_INVALID_ARG
    assert L.sw_server_fixed_bytes(None) == 0

def test_misaligned_offsets_rejected_on_host():
    # device offsets are read with 16-byte loads from the aligned address
    # below them: an array that does not start on 4 bytes is refused before
    # any device call, by every entry point that takes one
    import paper_1411_5283_amd as sw
    if not os.path.exists(sw.LIB_PATH):
        pytest.skip("library not built")
    L = sw.lib()
    buf = ctypes.create_string_buffer(256)
    p = (ctypes.addressof(buf) + 15) & ~15
    m = p + 2                                   # misaligned
    big = 1 << 30
    calls = {
        "sort_words": lambda o: L.sort_words(p, o, 3, p, p),
        "sort_words_ex": lambda o: L.sort_words_ex(p, o, 3, p, p, p, big, None),
        "sort_words_noalloc": lambda o: L.sort_words_noalloc(p, o, 3, p, p, p, None),
        "sort_words_batch": lambda o: L.sort_words_batch(p, o, p, 1, p, p, p, big, None),
        "sort_words_batch docs": lambda o: L.sort_words_batch(p, p, o, 1, p, p, p, big, None),
        "sort_words_plain": lambda o: L.sort_words_plain(p, o, p, 1, p, p, p, big, None),
        "sort_words_chunks": lambda o: L.sort_words_chunks(p, o, 3, 16, p, p, p, big, None),
        "sort_words_unbucketed": lambda o: L.sort_words_unbucketed(p, o, 3, p, p, p, big, None),
        "sort_words_materialize": lambda o: L.sort_words_materialize(p, o, None, 1, 3, p, p, 10, p, p, None),
    }
    for name, call in calls.items():
        assert call(m) == sw.ERR_INVALID_ARG, name
        assert b"aligned" in L.sort_words_last_error(), name
