// sw_window.hpp -- the step bookkeeping of the four-way merge pass by bounded
// windows (k_merge4w in sw_kernels.hpp), as plain code built for the device
// and, by its test, for the host.
//
// A four-way pass merges groups of four consecutive sorted runs into one run:
// two doublings of the run length for one HBM read and one write of every
// item.  A workgroup walks a contiguous range of the pass's output in steps.
// At a step every run shows a window of its next W unconsumed items; a window
// is full when its run goes on past it.  Let b be the smallest last item of a
// full window.  Every unconsumed item at or below b lies in a window (a full
// window ends at or above b, and a window that is not full holds the rest of
// its run), so the window items at or below b are exactly the next items of
// the merged order: the step consumes them (at least the W of b's own window;
// everything left when no window is full), merges them in LDS as
// merge(merge(A, B), merge(C, D)) and writes them out.  The next step's
// windows start where these counts end, and their loads are issued while
// this step merges.  Only the window items above b are read again at the next
// step, so a step reads its HBM bytes once plus about that tail from cache,
// and no ring or per-step search in HBM is needed.
#pragma once

#include <stdint.h>

namespace sw {

// Four-way pass geometry of a segment of n items whose runs hold R items:
// the group of four runs holding segment position s, its runs (start inside
// the group, length) and the rank of s inside the group.  The last group of a
// segment may hold fewer or shorter runs (empty runs have length 0).
struct M4Group {
  uint64_t start;       // group's first position in the segment
  uint32_t run_off[4];  // runs' first positions relative to the group
  uint32_t len[4];
  uint32_t size;        // items in the group
  uint32_t d;           // rank of s inside the group
};
__host__ __device__ inline M4Group m4_group(uint32_t n, uint64_t s, uint64_t R) {
  M4Group g;
  const uint64_t G = 4 * R;
  g.start = (s / G) * G;
  g.d = (uint32_t)(s - g.start);
  uint64_t at = g.start;
  for (int i = 0; i < 4; ++i) {
    g.run_off[i] = (uint32_t)(at - g.start);
    const uint64_t e = at + R < n ? at + R : (uint64_t)n;
    g.len[i] = e > at ? (uint32_t)(e - at) : 0u;
    at = e > at ? e : at;
  }
  g.size = (uint32_t)(at - g.start);
  return g;
}

constexpr int kWinRuns = 4;
constexpr uint32_t kWinLanes = 64;   // lanes of the slice search (one wave)

// Items in run r's window: its next W unconsumed items, or what is left.
__host__ __device__ inline uint32_t win_len(uint32_t len, uint32_t cons, uint32_t W) {
  const uint32_t left = len - cons;
  return left < W ? left : W;
}
// Whether the run goes on past its window.
__host__ __device__ inline bool win_full(uint32_t len, uint32_t cons, uint32_t W) { return len - cons > W; }

// The bounding run: the full window whose last item is smallest, or -1 when
// no window is full (then every window is taken whole).  last(r) reads item
// W-1 of run r's window; less is the strict order of the keys.
template <class K, class Last, class Less>
__host__ __device__ inline int win_bound(const uint32_t (&len)[kWinRuns], const uint32_t (&cons)[kWinRuns],
                                         uint32_t W, Last last, Less less, K& bound) {
  int br = -1;
  for (int r = 0; r < kWinRuns; ++r) {
    if (!win_full(len[r], cons[r], W)) continue;
    const K v = last(r);
    if (br < 0 || less(v, bound)) {
      br = r;
      bound = v;
    }
  }
  return br;
}

// Items of a sorted window of n <= 64*64 items below the bound, by two rounds
// of 64 probes: slice width s = ceil(n/64); in round 1 lane j probes the last
// item of slice j (when the slice lies inside the window), and k lanes find
// theirs below, so the count lies in slice k; in round 2 lane j < s probes
// item k*s + j.  The count is k*s plus the lanes below in round 2.
__host__ __device__ inline uint32_t win_slice(uint32_t n) { return (n + kWinLanes - 1) / kWinLanes; }
// Round 1: the item lane j probes, or -1.
__host__ __device__ inline int win_probe1(uint32_t n, uint32_t j) {
  const uint32_t s = win_slice(n);
  return (j + 1) * s <= n ? (int)((j + 1) * s - 1) : -1;
}
// Round 2, after k lanes were below in round 1: the item lane j probes, or -1.
__host__ __device__ inline int win_probe2(uint32_t n, uint32_t k, uint32_t j) {
  const uint32_t s = win_slice(n), i = k * s + j;
  return j < s && i < n ? (int)i : -1;
}

// Step counts: c[r] items of each window are consumed, given the bounding
// run br (-1: none) and, for every other run, the number of its window's
// items below the bound (below[r]; ignored when br < 0).
__host__ __device__ inline void win_counts(const uint32_t (&len)[kWinRuns], const uint32_t (&cons)[kWinRuns],
                                           uint32_t W, int br, const uint32_t (&below)[kWinRuns],
                                           uint32_t (&c)[kWinRuns]) {
  for (int r = 0; r < kWinRuns; ++r)
    c[r] = br < 0 ? win_len(len[r], cons[r], W) : (r == br ? W : below[r]);
}

// Which window item thread t's u-th load fetches when NT threads load the four
// windows of W = NT*E/4 items, E loads a thread: item q = t + u*NT, run q / W,
// position q % W.  With W a multiple of 64 every wave's u-th load stays inside
// one run.
__host__ __device__ inline int win_load_run(int u, int t, int NT, int W) { return (t + u * NT) / W; }
__host__ __device__ inline int win_load_pos(int u, int t, int NT, int W) { return (t + u * NT) % W; }

}  // namespace sw
