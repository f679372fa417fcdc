"""Result checks that hold at any size (invariants of a correct word sort).

Used by the CPU oracle tests and by the GPU parity tests on inputs too large
for the oracle to sort whole.
"""
import numpy as np

MAX_LEN = 32
N_OFFSETS = MAX_LEN + 2


def lengths(offsets):
    o = np.asarray(offsets, dtype=np.int64)
    return o[1:] - o[:-1]


def padded_bytes(chars, offsets, width=None):
    """[n, width] uint8 matrix of the words, zero padded on the right."""
    o = np.asarray(offsets, dtype=np.int64)
    lens = o[1:] - o[:-1]
    n = lens.shape[0]
    width = int(lens.max()) if (width is None and n) else (width or 0)
    M = np.zeros((n, max(width, 1)), np.uint8)
    if n == 0 or width == 0:
        return M
    start = o[:-1] - int(o[0])
    ch = np.asarray(chars)[int(o[0]):int(o[-1])]
    for j in range(width):
        has = lens > j
        M[has, j] = ch[start[has] + j]
    return M


def check_invariants(chars, offsets, perm, boff):
    """I1..I5: permutation, strictly increasing key (length, bytes, index),
    bucket sizes equal the length histogram, words sit in their length's
    bucket, offsets start at 0, do not decrease and end at n."""
    perm = np.asarray(perm, dtype=np.int64)
    boff = np.asarray(boff, dtype=np.int64)
    lens = lengths(offsets)
    n = lens.shape[0]
    assert perm.shape[0] == n
    assert boff.shape[0] == N_OFFSETS
    # I1
    if n:
        assert perm.min() >= 0 and perm.max() < n
        assert np.all(np.bincount(perm, minlength=n) == 1), "not a permutation"
    # I5
    assert boff[0] == 0 and boff[-1] == n and np.all(np.diff(boff) >= 0)
    # I3
    hist = np.bincount(lens, minlength=MAX_LEN + 1)[:MAX_LEN + 1]
    assert np.array_equal(np.diff(boff), hist), "bucket sizes differ from the length histogram"
    # I4
    pl = lens[perm] if n else lens
    for L in range(MAX_LEN + 1):
        assert np.all(pl[boff[L]:boff[L + 1]] == L)
    # I2: compare neighbours column by column, 8 bytes (big-endian) at a time
    if n > 1:
        width = int(lens.max())
        M = padded_bytes(chars, offsets, width=-(-max(width, 1) // 8) * 8)
        cols = M.view(">u8")
        a, b = perm[:-1], perm[1:]
        la, lb = lens[a], lens[b]
        lt = la < lb
        eq = la == lb
        for j in range(cols.shape[1]):
            ca, cb = cols[a, j], cols[b, j]
            lt |= eq & (ca < cb)
            eq &= ca == cb
        lt |= eq & (a < b)
        assert np.all(lt), "key order violated at %d places" % int((~lt).sum())
