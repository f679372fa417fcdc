// The four-run co-rank search (csrc/sw_split.hpp, the code the merge kernel
// runs with one thread per slot) driven on the host slot by slot, checked
// against the co-ranks read off a plain merge of the runs: every rank of
// small runs of many shapes, random ranks of runs up to 2^20 items, empty
// runs, and a bound on the number of rounds.  Prints "OK" and exits 0, or
// names the failing case and exits 1.
#define __host__
#define __device__
#include "sw_split.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using Key = uint64_t;

#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      std::printf("FAIL line %d: ", __LINE__); \
      std::printf(__VA_ARGS__);                \
      std::printf("\n");                       \
      std::exit(1);                            \
    }                                          \
  } while (0)

struct LessKey {
  bool operator()(const Key& a, const Key& b) const { return a < b; }
};

// The search as the kernel runs it: every slot loads its item, every interior
// slot gives its verdict, the brackets narrow; returns the rounds taken.
static int search(const std::vector<Key> (&runs)[4], uint32_t d, uint32_t (&s)[4]) {
  static sw::SplitScratch<Key> sc;   // large: kept off the stack
  uint32_t len[4];
  for (int i = 0; i < 4; ++i) len[i] = (uint32_t)runs[i].size();
  sw::split_init(sc, len, d);
  while (!sc.done) {
    CHECK(sc.rounds < (uint32_t)sw::kSplitMaxRounds, "no convergence, d=%u", d);
    sw::split_begin_round(sc);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < sw::kSplitSlots; ++j) {
        const uint32_t p = sw::split_slot_pos(sc, i, j);
        sc.pos[i][j] = p;
        if (p != sw::kSplitNone) {
          CHECK(p < len[i], "slot %d of run %d reads position %u of %u", j, i, p, len[i]);
          sc.key[i][j] = runs[i][p];
        }
      }
    for (int i = 0; i < 4; ++i)
      for (int j = 1; j + 1 < sw::kSplitSlots; ++j) {
        if (sc.pos[i][j] == sw::kSplitNone) continue;
        const int v = sw::split_decide(sc, i, j, LessKey());
        if (v < 0) sc.newlo[i] = std::max(sc.newlo[i], sc.pos[i][j] + 1);
        if (v > 0) sc.newhi[i] = std::min(sc.newhi[i], sc.pos[i][j]);
      }
    for (int i = 0; i < 4; ++i) CHECK(sc.newlo[i] <= sc.newhi[i], "bracket of run %d crossed, d=%u", i, d);
    sw::split_finish_round(sc);
  }
  for (int i = 0; i < 4; ++i) s[i] = sc.lo[i];
  return (int)sc.rounds;
}

// Co-ranks read off the merged order: how many of the first d come from each
// run, for every d (a plain merge, then prefix counts).
struct Expected {
  std::vector<uint8_t> from;   // run of the k-th smallest item
  void build(const std::vector<Key> (&runs)[4]) {
    std::vector<std::pair<Key, int>> all;
    for (int i = 0; i < 4; ++i)
      for (Key k : runs[i]) all.push_back({k, i});
    std::sort(all.begin(), all.end());
    from.resize(all.size());
    for (size_t k = 0; k < all.size(); ++k) from[k] = (uint8_t)all[k].second;
  }
  void at(uint32_t d, uint32_t (&s)[4]) const {
    for (int i = 0; i < 4; ++i) s[i] = 0;
    for (uint32_t k = 0; k < d; ++k) s[from[k]] += 1;
  }
};

// Four sorted runs of distinct keys: `shape` picks how the runs interleave.
static void make_runs(std::mt19937_64& rng, const uint32_t (&len)[4], int shape, std::vector<Key> (&runs)[4]) {
  uint32_t total = 0;
  for (int i = 0; i < 4; ++i) total += len[i];
  std::vector<Key> keys(total);
  // distinct keys: a random permutation of a spread-out range
  for (uint32_t k = 0; k < total; ++k) keys[k] = (Key)k * 7919u + 13u;
  std::shuffle(keys.begin(), keys.end(), rng);
  if (shape == 1) std::sort(keys.begin(), keys.end());                  // runs in disjoint key ranges
  if (shape == 2) std::sort(keys.begin(), keys.end(), std::greater<Key>());   // disjoint, reversed
  if (shape == 3) {                                                     // long stretches from one run
    std::sort(keys.begin(), keys.end());
    for (uint32_t a = 0; a < total; a += 97) std::reverse(keys.begin() + a, keys.begin() + std::min(total, a + 97));
  }
  uint32_t at = 0;
  for (int i = 0; i < 4; ++i) {
    runs[i].assign(keys.begin() + at, keys.begin() + at + len[i]);
    std::sort(runs[i].begin(), runs[i].end());
    at += len[i];
  }
}

int main() {
  std::mt19937_64 rng(1411);
  // 1. every rank of small runs, many shapes and lengths (empty runs included)
  const uint32_t small_lens[][4] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {0, 0, 0, 5}, {3, 3, 3, 3},   {1, 2, 3, 4},
                                    {62, 62, 62, 62}, {63, 1, 0, 70}, {100, 0, 100, 0}, {200, 7, 130, 64},
                                    {500, 500, 1, 1}, {61, 62, 63, 64}, {2, 300, 2, 300}};
  for (const auto& L : small_lens)
    for (int shape = 0; shape < 4; ++shape) {
      std::vector<Key> runs[4];
      make_runs(rng, L, shape, runs);
      const uint32_t total = L[0] + L[1] + L[2] + L[3];
      Expected ex;
      ex.build(runs);
      for (uint32_t d = 0; d <= total; ++d) {
        uint32_t got[4], exp[4];
        search(runs, d, got);
        ex.at(d, exp);
        for (int i = 0; i < 4; ++i)
          CHECK(got[i] == exp[i], "lens %u %u %u %u shape %d d=%u run %d: %u, expected %u", L[0], L[1], L[2], L[3],
                shape, d, i, got[i], exp[i]);
      }
    }
  // 2. random lengths and ranks, larger runs; rounds stay few
  int max_rounds = 0;
  for (int t = 0; t < 124; ++t) {
    uint32_t L[4];
    const uint32_t cap = t < 100 ? 5000 : (1u << 20);
    for (int i = 0; i < 4; ++i) L[i] = (rng() % 4 == 0) ? (uint32_t)(rng() % 3) : (uint32_t)(rng() % cap);
    if (t >= 122)
      for (int i = 0; i < 4; ++i) L[i] = 1u << 20;   // equal full runs, as in a top merge level
    std::vector<Key> runs[4];
    make_runs(rng, L, (int)(rng() % 4), runs);
    const uint64_t total = (uint64_t)L[0] + L[1] + L[2] + L[3];
    Expected ex;
    ex.build(runs);
    for (int k = 0; k < 8; ++k) {
      const uint32_t d = k == 0 ? 0u : (k == 1 ? (uint32_t)total : (uint32_t)(rng() % (total + 1)));
      uint32_t got[4], exp[4];
      const int r = search(runs, d, got);
      max_rounds = std::max(max_rounds, r);
      ex.at(d, exp);
      for (int i = 0; i < 4; ++i)
        CHECK(got[i] == exp[i], "random case %d d=%u run %d: %u, expected %u", t, d, i, got[i], exp[i]);
    }
  }
  // brackets shrink by about 62/5 a round: four runs of 2^20 need at most 6
  CHECK(max_rounds <= 7, "a search took %d rounds", max_rounds);
  std::printf("max rounds %d\nOK\n", max_rounds);
  return 0;
}
