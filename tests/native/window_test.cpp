// The four-way merge pass by bounded windows (csrc/sw_window.hpp, the step
// bookkeeping k_merge4w runs) driven on the host: groups of four sorted runs
// of many shapes (empty, short, equal, disjoint, interleaved, one run far
// below the others), windows of 16..4096 items, and every step of the walk
// from a random start rank:
//  * the bounding run and the counts (the slice search emulated lane by lane)
//    equal their definitions: the window items at or below the bound;
//  * those items are exactly the next items of the merged order (against a
//    plain sort of the group), so the merged walk reproduces it;
//  * a step takes at least W items unless it takes everything left, at most
//    4W, and every window read and sentinel slot lies inside its run and its
//    W+1 slots;
//  * the window loads of NT threads, E items each, cover every window slot
//    once, each wave's load inside one run.
// Prints "OK" and exits 0, or names the failing case and exits 1.
#define __host__
#define __device__
#include "sw_window.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      std::printf("FAIL line %d: ", __LINE__); \
      std::printf(__VA_ARGS__);                \
      std::printf("\n");                       \
      std::exit(1);                            \
    }                                          \
  } while (0)

using Runs = std::vector<std::vector<uint64_t>>;

// four runs of distinct keys in one of several shapes
static Runs make_group(std::mt19937_64& rng, int shape, uint32_t maxlen) {
  Runs runs(4);
  uint32_t len[4];
  for (int r = 0; r < 4; ++r) {
    const uint32_t pick = (uint32_t)(rng() % 6);
    len[r] = pick == 0 ? 0u : (pick == 1 ? 1u + (uint32_t)(rng() % 8) : (uint32_t)(rng() % (maxlen + 1)));
  }
  if (shape == 1)
    for (int r = 1; r < 4; ++r) len[r] = len[0];
  std::vector<uint64_t> keys;
  const uint32_t total = len[0] + len[1] + len[2] + len[3];
  while (keys.size() < total) keys.push_back(rng() >> 8);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  while (keys.size() < total) keys.push_back(keys.empty() ? 1 : keys.back() + 1 + (rng() % 5));
  std::shuffle(keys.begin(), keys.end(), rng);
  size_t at = 0;
  for (int r = 0; r < 4; ++r) {
    runs[r].assign(keys.begin() + at, keys.begin() + at + len[r]);
    at += len[r];
    std::sort(runs[r].begin(), runs[r].end());
  }
  if (shape == 2) {
    // disjoint ranges: run r's keys all below run r+1's
    std::vector<uint64_t> all = keys;
    std::sort(all.begin(), all.end());
    at = 0;
    for (int r = 0; r < 4; ++r) {
      runs[r].assign(all.begin() + at, all.begin() + at + len[r]);
      at += len[r];
    }
  }
  if (shape == 3 && total > 0) {
    // run 3 far below the rest
    for (auto& v : runs[3]) v >>= 20;
    std::vector<uint64_t> u;
    for (auto& rr : runs) u.insert(u.end(), rr.begin(), rr.end());
    std::sort(u.begin(), u.end());
    if (std::adjacent_find(u.begin(), u.end()) != u.end()) return make_group(rng, 0, maxlen);
  }
  return runs;
}

static void walk(std::mt19937_64& rng, const Runs& runs, uint32_t W) {
  uint32_t len[4];
  std::vector<std::pair<uint64_t, int>> all;
  for (int r = 0; r < 4; ++r) {
    len[r] = (uint32_t)runs[r].size();
    for (uint64_t v : runs[r]) all.push_back({v, r});
  }
  std::sort(all.begin(), all.end());
  const uint32_t total = (uint32_t)all.size();
  const uint32_t d0 = total ? (uint32_t)(rng() % (total + 1)) : 0u;
  // start co-ranks from the definition (the split search's result)
  uint32_t cons[4] = {0, 0, 0, 0};
  for (uint32_t i = 0; i < d0; ++i) cons[all[i].second]++;
  std::vector<uint64_t> out;
  auto less = [](uint64_t a, uint64_t b) { return a < b; };
  int steps = 0;
  while (out.size() + d0 < total) {
    CHECK(++steps <= (int)total + 2, "W=%u: no progress", W);
    // the windows, W+1 slots each (a sentinel slot after the items)
    std::vector<uint64_t> win[4];
    uint32_t wl[4];
    for (int r = 0; r < 4; ++r) {
      wl[r] = sw::win_len(len[r], cons[r], W);
      CHECK(wl[r] <= W && cons[r] + wl[r] <= len[r], "window leaves run %d", r);
      win[r].assign(runs[r].begin() + cons[r], runs[r].begin() + cons[r] + wl[r]);
    }
    uint64_t bound = ~0ull;
    const int br = sw::win_bound(len, cons, W, [&](int r) { return win[r][W - 1]; }, less, bound);
    // the bound by its definition
    int want_br = -1;
    uint64_t want_b = 0;
    for (int r = 0; r < 4; ++r)
      if (len[r] - cons[r] > W && (want_br < 0 || win[r][W - 1] < want_b)) {
        want_br = r;
        want_b = win[r][W - 1];
      }
    CHECK(br == want_br && (br < 0 || bound == want_b), "W=%u: bounding run %d, expected %d", W, br, want_br);
    // each run's items below the bound, by the two probe rounds of 64 lanes
    uint32_t below[4] = {0, 0, 0, 0};
    for (int r = 0; r < 4; ++r) {
      if (br < 0 || r == br) continue;
      uint32_t k1 = 0;
      for (uint32_t j = 0; j < sw::kWinLanes; ++j) {
        const int p = sw::win_probe1(wl[r], j);
        CHECK(p < (int)wl[r], "round 1 probe %d outside a window of %u", p, wl[r]);
        k1 += (p >= 0 && win[r][p] < bound) ? 1u : 0u;
      }
      uint32_t k2 = 0;
      for (uint32_t j = 0; j < sw::kWinLanes; ++j) {
        const int p = sw::win_probe2(wl[r], k1, j);
        CHECK(p < (int)wl[r], "round 2 probe %d outside a window of %u", p, wl[r]);
        k2 += (p >= 0 && win[r][p] < bound) ? 1u : 0u;
      }
      below[r] = k1 * sw::win_slice(wl[r]) + k2;
      const uint32_t want =
          (uint32_t)(std::lower_bound(win[r].begin(), win[r].end(), bound) - win[r].begin());
      CHECK(below[r] == want, "W=%u run %d: %u below the bound, expected %u", W, r, below[r], want);
    }
    uint32_t c[4];
    sw::win_counts(len, cons, W, br, below, c);
    uint32_t ns = 0;
    for (int r = 0; r < 4; ++r) {
      CHECK(c[r] <= wl[r] && c[r] <= W, "count %u of a window of %u", c[r], wl[r]);   // sentinel slot c <= W
      ns += c[r];
    }
    const uint32_t left = total - d0 - (uint32_t)out.size();
    CHECK(ns <= 4 * W, "step of %u items over 4W", ns);
    CHECK(ns >= W || ns == left, "W=%u: step of %u items with %u left", W, ns, left);
    // merge(merge(A, B), merge(C, D)) of the counted items
    std::vector<uint64_t> X, Y, Z;
    std::merge(win[0].begin(), win[0].begin() + c[0], win[1].begin(), win[1].begin() + c[1], std::back_inserter(X));
    std::merge(win[2].begin(), win[2].begin() + c[2], win[3].begin(), win[3].begin() + c[3], std::back_inserter(Y));
    std::merge(X.begin(), X.end(), Y.begin(), Y.end(), std::back_inserter(Z));
    for (size_t i = 0; i < Z.size(); ++i)
      CHECK(Z[i] == all[d0 + out.size() + i].first, "W=%u step %d: output %zu is not the merged order", W, steps, i);
    out.insert(out.end(), Z.begin(), Z.end());
    for (int r = 0; r < 4; ++r) cons[r] += c[r];
  }
  CHECK(out.size() + d0 == total, "walk ended with %zu of %u", out.size() + d0, total);
}

// the window loads of NT threads, E items a thread
static void check_loads(int NT, int E) {
  const int W = NT * E / 4;
  std::vector<int> hits(4 * W, 0);
  for (int u = 0; u < E; ++u)
    for (int t = 0; t < NT; ++t) {
      const int r = sw::win_load_run(u, t, NT, W), i = sw::win_load_pos(u, t, NT, W);
      CHECK(r >= 0 && r < 4 && i >= 0 && i < W, "NT=%d E=%d u=%d t=%d: run %d position %d", NT, E, u, t, r, i);
      CHECK(r == sw::win_load_run(u, t & ~63, NT, W), "NT=%d E=%d u=%d: a wave's load crosses runs", NT, E, u);
      hits[r * W + i]++;
    }
  for (int q = 0; q < 4 * W; ++q) CHECK(hits[q] == 1, "NT=%d E=%d: slot %d loaded %d times", NT, E, q, hits[q]);
}

int main() {
  std::mt19937_64 rng(5283);
  int groups = 0;
  for (uint32_t W : {16u, 64u, 100u, 256u, 512u, 1024u, 4096u})
    for (int rep = 0; rep < 120; ++rep, ++groups) {
      const uint32_t maxlen = rep < 60 ? 3 * W : 20 * W;
      walk(rng, make_group(rng, rep % 4, maxlen), W);
    }
  for (int NT : {256, 512, 1024})
    for (int E : {1, 2, 4, 8, 12, 16}) check_loads(NT, E);
  std::printf("window groups walked: %d\nOK\n", groups);
  return 0;
}
