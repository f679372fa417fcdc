// sw_split.hpp -- exact co-ranks of one rank in four sorted runs, as plain
// integer code built for the device and, by its tests, for the host.
//
// Problem: runs S_0..S_3 (sorted, every key distinct across all of them) and a
// rank d; find s_i, the number of items of run i among the d smallest of the
// union (sum of s_i = d).  Merge path gives this for two runs with one binary
// search; for four there is no single monotone diagonal, so the search keeps
// a bracket [lo_i, hi_i] that holds s_i for every run and shrinks all four
// together.  A round samples each bracket at up to 62 evenly spaced
// positions, plus the item just before the bracket (known to be among the d
// smallest) and the item at its end (known not to be).  For a sample y of run
// i at position q, rank(y) = q + sum over the other runs of #{items < y}; each
// of those counts lies between two neighbouring samples of that run (or is
// decided outright when y falls outside the other bracket's known items), so
// rank(y) is known to within about one sample spacing per run.  A sample
// whose rank is surely below d lifts lo_i past it, one surely at or above d
// lowers hi_i to it.  The largest bracket shrinks by about 62/5 per round;
// once every bracket holds at most 62 items every position is sampled, every
// rank is exact and the brackets close.
//
// The scratch below is shared by the workgroup (LDS) on the device and is an
// ordinary struct on the host; the sampling (one thread per slot) and the
// decisions (one thread per interior slot) are the same functions on both.
#pragma once

#include <stdint.h>

namespace sw {

constexpr int kSplitRuns = 4;
constexpr int kSplitSlots = 64;      // per run: boundary below, 62 interior, boundary at the end
constexpr int kSplitInterior = kSplitSlots - 2;
constexpr int kSplitMaxRounds = 40;  // far above what any run of 2^32 items needs
constexpr uint32_t kSplitNone = 0xFFFFFFFFu;

template <class K>
struct SplitScratch {
  K key[kSplitRuns][kSplitSlots];
  uint32_t pos[kSplitRuns][kSplitSlots];   // kSplitNone: slot unused this round
  uint64_t start[kSplitRuns];               // where each run's item 0 is (for the caller's loads)
  uint32_t len[kSplitRuns], lo[kSplitRuns], hi[kSplitRuns];
  uint32_t newlo[kSplitRuns], newhi[kSplitRuns];
  uint32_t d, done, rounds;
};

// Start of a search (one thread): brackets from the lengths alone.
template <class K>
__host__ __device__ __attribute__((always_inline)) inline void split_init(SplitScratch<K>& s, const uint32_t (&len)[kSplitRuns], uint32_t d) {
  uint64_t total = 0;
  for (int i = 0; i < kSplitRuns; ++i) total += len[i];
  for (int i = 0; i < kSplitRuns; ++i) {
    const uint64_t others = total - len[i];
    s.len[i] = len[i];
    s.lo[i] = d > others ? (uint32_t)(d - others) : 0u;
    s.hi[i] = d < len[i] ? d : len[i];
  }
  s.d = d;
  s.rounds = 0;
  bool done = true;
  for (int i = 0; i < kSplitRuns; ++i) done = done && s.lo[i] == s.hi[i];
  s.done = done ? 1u : 0u;
}

// Position of interior sample jj (0..61) of a bracket, or kSplitNone.  Wider
// brackets are sampled at floor(jj * w / 62): strictly increasing in jj.
__host__ __device__ __attribute__((always_inline)) inline uint32_t split_sample_pos(uint32_t lo, uint32_t hi, uint32_t jj) {
  const uint32_t w = hi - lo;
  if (w <= (uint32_t)kSplitInterior) return jj < w ? lo + jj : kSplitNone;
  return lo + (uint32_t)(((uint64_t)jj * w) / (uint32_t)kSplitInterior);
}

// The run position slot j of run i reads this round, or kSplitNone: slot 0 is
// the item just below the bracket (among the d smallest), slot 63 the item at
// the bracket's end (not among them), slots 1..62 the interior samples.
template <class K>
__host__ __device__ __attribute__((always_inline)) inline uint32_t split_slot_pos(const SplitScratch<K>& s, int i, int j) {
  if (j == 0) return s.lo[i] > 0 ? s.lo[i] - 1 : kSplitNone;
  if (j == kSplitSlots - 1) return s.hi[i] < s.len[i] ? s.hi[i] : kSplitNone;
  return split_sample_pos(s.lo[i], s.hi[i], (uint32_t)(j - 1));
}

// Interior samples of run i this round (slots 1..n).
template <class K>
__host__ __device__ __attribute__((always_inline)) inline uint32_t split_interior(const SplitScratch<K>& s, int i) {
  const uint32_t w = s.hi[i] - s.lo[i];
  return w < (uint32_t)kSplitInterior ? w : (uint32_t)kSplitInterior;
}

// Verdict on interior slot j (1..62, in use) of run i: -1 when its item is
// surely among the d smallest, +1 when surely not, 0 when the samples cannot
// tell yet.  `less` is the strict order of the keys.
template <class K, class Less>
__host__ __device__ __attribute__((always_inline)) inline int split_decide(const SplitScratch<K>& s, int i, int j, Less less) {
  const K& y = s.key[i][j];
  const uint32_t q = s.pos[i][j];
  uint64_t rlo = q, rhi = q;   // bounds of rank(y) = number of items below y
  for (int o = 0; o < kSplitRuns; ++o) {
    if (o == i) continue;
    // below the item just under run o's bracket: below the d-th item
    if (s.lo[o] > 0 && less(y, s.key[o][0])) return -1;
    // above the item at run o's bracket end: above it too
    if (s.hi[o] < s.len[o] && less(s.key[o][kSplitSlots - 1], y)) return 1;
    // y lies inside run o's bracket: count run o's interior samples below y
    const uint32_t n = split_interior(s, o);
    uint32_t a = 0, b = n;
    while (a < b) {
      const uint32_t m = (a + b) >> 1;
      if (less(s.key[o][1 + m], y))
        a = m + 1;
      else
        b = m;
    }
    rlo += a > 0 ? s.pos[o][a] + 1 : s.lo[o];          // sample a-1 (slot a) is below y
    rhi += a < n ? s.pos[o][1 + a] : s.hi[o];          // sample a (slot a+1) is above y
  }
  if (rhi < s.d) return -1;
  if (rlo >= s.d) return 1;
  return 0;
}

// End of a round (one thread, after every verdict has been applied to
// newlo/newhi): the new brackets, and whether they have closed.
template <class K>
__host__ __device__ __attribute__((always_inline)) inline void split_finish_round(SplitScratch<K>& s) {
  bool done = true;
  for (int i = 0; i < kSplitRuns; ++i) {
    s.lo[i] = s.newlo[i];
    s.hi[i] = s.newhi[i];
    done = done && s.lo[i] == s.hi[i];
  }
  s.rounds += 1;
  s.done = done ? 1u : 0u;
}

// Start of a round (one thread): the verdicts narrow from the current brackets.
template <class K>
__host__ __device__ __attribute__((always_inline)) inline void split_begin_round(SplitScratch<K>& s) {
  for (int i = 0; i < kSplitRuns; ++i) {
    s.newlo[i] = s.lo[i];
    s.newhi[i] = s.hi[i];
  }
}

}  // namespace sw
