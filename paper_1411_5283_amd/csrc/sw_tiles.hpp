// sw_tiles.hpp -- geometry of the two-way merge levels (which runs a merge
// tile reads, where it writes, how a workgroup's tiles are placed), as plain
// integer code built for the device and, by its tests, for the host.
//
// A segment of n items after the chunk sort holds sorted runs of T items; at
// merge level l the runs hold R = T << l items and pairs of neighbouring
// runs (A, then B) are merged into runs of 2R.  The level's outputs are cut
// into merge tiles of P items (P and R powers of two, P <= 2T); tile j's
// outputs are positions [jP, jP + P) of the segment, inside one pair.  Merge
// path (Odeh et al., IPDPSW 2012): the first d outputs of merging A and B are
// A[0, s) and B[0, d - s) for one split s, and the tile's inputs are the A
// and B items between its first and its last output's splits.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace sw {

__host__ __device__ __attribute__((always_inline)) inline uint32_t tmin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__host__ __device__ __attribute__((always_inline)) inline int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ __attribute__((always_inline)) inline int imax(int a, int b) { return a > b ? a : b; }

// Merge levels of a segment of n items after tiles of T = 2^lt: the smallest
// m with T*2^m >= n is ceil(log2 n) - lt (at least 0), and ceil(log2 n) is
// the bit length of n-1.
__host__ __device__ inline uint32_t levels_pow2(uint32_t n, uint32_t lt) {
  if (n <= 1) return 0;
  const uint32_t bits = 32u - (uint32_t)__builtin_clz(n - 1);
  return bits > lt ? bits - lt : 0u;
}

// Geometry of merge tile j (P outputs) of a segment of n items at a level
// whose runs hold R items: the pair start ps, the pair's run lengths la and
// lb, and the tile's diagonal range [d0, d1) inside the pair.
struct MergeTile {
  uint64_t o0, ps;
  uint32_t la, lb, d0, d1;
};
// R and P are powers of two, so the pair start is a mask, not a division.
__host__ __device__ inline MergeTile merge_tile(uint32_t n, uint32_t j, uint64_t R, uint32_t P) {
  MergeTile m;
  m.o0 = (uint64_t)j * P;
  m.ps = m.o0 & ~(2 * R - 1);
  const uint32_t rem = n - (uint32_t)m.ps;
  m.la = (uint32_t)(rem < R ? (uint64_t)rem : R);
  m.lb = rem - m.la < R ? rem - m.la : (uint32_t)R;
  m.d0 = (uint32_t)(m.o0 - m.ps);
  m.d1 = tmin(m.d0 + P, m.la + m.lb);
  return m;
}

// Placement of a merge tile: its segment (first position, size), its index in
// the segment, and the merge-path split at its first output (A items before
// it).
struct TileRec {
  uint32_t base, n, j, split;
};

// Where a merge tile reads and writes, from its placement and the split at
// its last output (the next tile's first split, or the pair's end).
struct TileIO {
  size_t apos, bpos, ob;
  int na, cnt;
  int final;   // nonzero on the segment's last level
};
__host__ __device__ inline TileIO tile_io(const TileRec& r, uint32_t end_split, uint64_t R, uint32_t P, uint32_t Tc,
                                          int level) {
  const MergeTile m = merge_tile(r.n, r.j, R, P);
  const uint32_t a1 = m.d1 == m.la + m.lb ? m.la : end_split;
  TileIO io;
  io.apos = (size_t)r.base + m.ps + r.split;
  io.bpos = (size_t)r.base + m.ps + m.la + (m.d0 - r.split);
  io.ob = (size_t)r.base + m.o0;
  // A items [split, a1), B items from d0 - split.  With both splits taken
  // by merge path on the same pair, max(0, d - lb) <= s(d) <= min(d, la) and
  // s is nondecreasing, so the counts below never clamp (the host test of
  // this file checks every tile of random segments); the clamps stay so that
  // splits from a damaged workspace read inside the pair's runs rather than
  // outside them.
  const int cnt = (int)(m.d1 - m.d0);
  const int a_left = (int)m.la - (int)r.split, b_left = (int)m.lb - (int)(m.d0 - r.split);
  io.na = imin(imax((int)a1 - (int)r.split, 0), imin(cnt, imax(a_left, 0)));
  io.cnt = io.na + imin(cnt - io.na, imax(b_left, 0));
  io.final = levels_pow2(r.n, (uint32_t)__builtin_ctz(Tc)) == (uint32_t)level + 1;
  return io;
}

// A workgroup of NG groups places tiles t0, t0+1, ... of its range [tb,
// t_end): group g takes tile t0 + g, and is active while that tile exists
// and is at most t_end (the tile one past the range is placed too: its first
// split is the range's last tile's end split).  Groups 0..NG-2 fill the
// records of NG-1 tiles; every active group gives its split.
__host__ __device__ inline bool place_group_active(uint32_t t0, uint32_t g, uint32_t ntiles, uint32_t t_end) {
  const uint32_t t = t0 + g;
  return t < ntiles && t <= t_end;
}
// The k-th tile of a range (k = 0, 1, ...) sits in batch slot k % (NG-1);
// a new batch is placed before tile k when k is a multiple of NG-1 (k > 0).
__host__ __device__ inline uint32_t place_slot(uint32_t k, uint32_t tiles_per_batch) { return k % tiles_per_batch; }

// One round of the K-ary search of a tile's segment: the last k in [lo, hi)
// with prefix[k] <= t (prefix[lo] <= t is known).  Lane gl of the group
// probes k = lo + gl*step; with c the number of lanes whose probe is <= t
// (c >= 1: lane 0 probes lo), the answer lies in [lo + (c-1)*step, that +
// step).  The device counts c with a ballot; the host test counts it in a
// loop.
struct KarySearch {
  uint32_t lo, hi;
  __host__ __device__ bool open() const { return hi - lo > 1; }
  __host__ __device__ uint32_t step(uint32_t K) const { return (hi - lo + K - 1) / K; }
  __host__ __device__ uint32_t probe(uint32_t gl, uint32_t K) const { return lo + gl * step(K); }
  __host__ __device__ void narrow(uint32_t c, uint32_t K) {
    const uint32_t s = step(K);
    const uint32_t nlo = lo + (c - 1) * s;
    hi = tmin(nlo + s, hi);
    lo = nlo;
  }
};

}  // namespace sw
