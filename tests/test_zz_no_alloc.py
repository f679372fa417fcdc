"""The entry point that allocates nothing (sort_words_noalloc) against the
workspace form (sort_words_ex) it is a variant of, through the C ABI: two
calls in a row on the one scratch, the second smaller, each equal to
sort_words_ex's result (and to the oracle's); the capacity limit and a
device-detected error come back as status codes."""
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


def _run_both(gpu, wl):
    import torch
    chars, offs, _ = gpu.device_words(wl, "cuda")
    n = wl.n
    perm_a = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    boff_a = torch.empty(34, dtype=torch.int32, device="cuda")
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    gpu.sort_words_noalloc(chars, offs, n, perm_a, boff_a, status)
    torch.cuda.synchronize()
    perm_b = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    boff_b = torch.empty(34, dtype=torch.int32, device="cuda")
    ws = torch.empty(gpu.sort_words_workspace_size(n, 1), dtype=torch.uint8, device="cuda")
    gpu.sort_words_ex(chars, offs, n, perm_b, boff_b, ws)
    gpu.sort_words_status(ws)
    return (int(status.cpu()[0]), gpu.to_u32(perm_a)[:n], gpu.to_u32(boff_a),
            gpu.to_u32(perm_b)[:n], gpu.to_u32(boff_b))


def test_noalloc_equals_workspace_form_twice(gpu, oracle_mod):
    lo, hi = 0, 1 << 22          # the largest n whose workspace fits the scratch
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if gpu.sort_words_workspace_size(mid, 1) <= gpu.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    cap = lo
    # the largest input that fits, then a smaller one on the same scratch
    big = wordgen.single(min(cap, 300_000), 20_000, 1.0, 32, seed=3)
    small = wordgen.config(1, 0.3)
    for rep, wl in enumerate((big, small, big)):
        _say("case noalloc call %d n=%d" % (rep, wl.n))
        st, pa, ba, pb, bb = _run_both(gpu, wl)
        assert gpu.decode_status(st) == gpu.OK and st == 0
        assert np.array_equal(pa, pb), "call %d: permutation differs from sort_words_ex" % rep
        assert np.array_equal(ba, bb), "call %d: bucket offsets differ from sort_words_ex" % rep
        ep, eb = oracle_mod.oracle_def(wl.chars, wl.offsets)
        assert np.array_equal(pa, ep) and np.array_equal(ba, eb), "call %d differs from the oracle" % rep


def test_noalloc_limits_and_errors(gpu):
    import torch
    _say("case noalloc limits")
    # above the scratch: refused at once, nothing enqueued
    n = 1
    while gpu.sort_words_workspace_size(n, 1) <= gpu.NOALLOC_SCRATCH_BYTES:
        n *= 2
    offs = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    boff = torch.empty(34, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.SortWordsError) as e:
        gpu.sort_words_noalloc(None, offs, n, perm, boff, status)
    assert e.value.code == gpu.ERR_WORKSPACE
    # a word too long: the device status word says so; the next call is clean
    chars = torch.zeros(64, dtype=torch.uint8, device="cuda")
    o = torch.tensor(np.asarray([0, 3, 40, 41], np.uint32).view(np.int32), device="cuda")
    gpu.sort_words_noalloc(chars, o, 3, perm, boff, status)
    torch.cuda.synchronize()
    assert gpu.decode_status(int(status.cpu()[0])) == gpu.ERR_WORD_TOO_LONG
    o = torch.tensor(np.asarray([0, 3, 5, 6], np.uint32).view(np.int32), device="cuda")
    gpu.sort_words_noalloc(chars, o, 3, perm, boff, status)
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == 0
