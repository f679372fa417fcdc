"""The register merge round of the chunk sort (lane_merge_round in
csrc/sw_kernels.hpp), emulated on the host with the kernel's index mapping:
lanes of E items each, pairs of runs of M*E items in 2M aligned lanes; the
first run's item i meets the second's mirror item (lane ^ (2M-1), item
E-1-r), the lower half keeping the smaller; for M = 2 a half-cleaner at lane
distance 1; then half-cleaners at item distance E/2 .. 1 inside each lane.
Afterwards every group of 2M lanes must hold its two runs merged, in blocked
order.  Checked for M = 1, 2 and E = 1..16 on random keys with duplicates,
on equal keys and on runs that do not interleave; a planted mistake (the
mirror taken as lane ^ 1 for M = 2) must fail."""
import numpy as np
import pytest


def lane_merge_round(lanes, M, mirror_xor=None):
    """lanes: array (64, E); returns the lanes after one round."""
    n, E = lanes.shape
    x = mirror_xor if mirror_xor is not None else 2 * M - 1
    out = lanes.copy()
    for l in range(n):
        upper = (l & M) != 0
        p = lanes[l ^ x]
        for r in range(E):
            q = p[E - 1 - r]
            take = (q < lanes[l, r]) != upper
            out[l, r] = q if take else lanes[l, r]
    if M == 2:
        cur = out.copy()
        for l in range(n):
            upper = (l & 1) != 0
            for r in range(E):
                q = cur[l ^ 1, r]
                out[l, r] = q if ((q < cur[l, r]) != upper) else cur[l, r]
    st = E // 2
    while st >= 1:
        for l in range(n):
            for i in range(E):
                if i & st == 0 and out[l, i] > out[l, i + st]:
                    out[l, i], out[l, i + st] = out[l, i + st], out[l, i]
        st //= 2
    return out


def _runs(rng, M, E, kind):
    lanes = np.empty((64, E), np.int64)
    R = M * E
    for g in range(0, 64, 2 * M):
        if kind == "random":
            a, b = np.sort(rng.integers(0, 50, R)), np.sort(rng.integers(0, 50, R))
        elif kind == "equal":
            a = b = np.full(R, 7)
        else:   # disjoint: every key of the first run above the second's
            b = np.sort(rng.integers(0, 100, R))
            a = np.sort(rng.integers(200, 300, R))
        lanes[g:g + 2 * M] = np.concatenate([a, b]).reshape(2 * M, E)
    return lanes


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("E", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("kind", ["random", "equal", "disjoint"])
def test_round_merges_each_pair(M, E, kind):
    rng = np.random.default_rng(M * 100 + E)
    for _ in range(3):
        lanes = _runs(rng, M, E, kind)
        got = lane_merge_round(lanes, M)
        for g in range(0, 64, 2 * M):
            want = np.sort(lanes[g:g + 2 * M].reshape(-1))
            assert np.array_equal(got[g:g + 2 * M].reshape(-1), want), (M, E, kind, g)


def test_planted_wrong_mirror_fails():
    rng = np.random.default_rng(5)
    bad = 0
    for _ in range(5):
        lanes = _runs(rng, 2, 4, "random")
        got = lane_merge_round(lanes, 2, mirror_xor=1)
        for g in range(0, 64, 4):
            bad += not np.array_equal(got[g:g + 4].reshape(-1), np.sort(lanes[g:g + 4].reshape(-1)))
    assert bad > 0
