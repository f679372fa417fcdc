// The two-way merge levels' tile geometry (csrc/sw_tiles.hpp, the code the
// merge kernel runs) driven on the host:
//  1. every tile of random segments at every level: the runs it reads lie
//     inside its pair, the counts never clamp, the inputs it merges are
//     exactly the outputs it owns (against a plain merge of the pair), the
//     tiles cover the segment once, and the last level is flagged;
//  2. the placement bookkeeping of a workgroup's range (batches of NG-1
//     records, the split of the tile one past each record): every tile of
//     every range gets its own record and its successor's split;
//  3. the K-ary search of a tile's segment in the class's tile prefix.
// Prints "OK" and exits 0, or names the failing case and exits 1.
#define __host__
#define __device__
#include "sw_tiles.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <numeric>
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

static uint32_t levels_for(uint32_t n, uint32_t T) {
  uint32_t m = 0;
  for (uint64_t r = T; r < n; r <<= 1) ++m;
  return m;
}

// 1. one segment of n distinct keys whose runs of R are sorted; every tile
static void check_level(std::mt19937_64& rng, uint32_t n, uint32_t T, uint32_t P, uint32_t level) {
  const uint64_t R = (uint64_t)T << level;
  std::vector<uint32_t> key(n);
  std::iota(key.begin(), key.end(), 0u);
  std::shuffle(key.begin(), key.end(), rng);
  for (uint64_t r = 0; r < n; r += R) std::sort(key.begin() + r, key.begin() + std::min<uint64_t>(n, r + R));
  const uint32_t base = (uint32_t)(rng() % 100000);
  // merged order of every pair, and the split (A items among the first d outputs) at every d
  std::vector<uint32_t> merged(n), split(n + 1);
  std::vector<uint32_t> split_at(n + 1);   // indexed by pair start + d
  for (uint64_t ps = 0; ps < n; ps += 2 * R) {
    const uint32_t la = (uint32_t)std::min<uint64_t>(R, n - ps), lb = (uint32_t)std::min<uint64_t>(R, n - ps - la);
    uint32_t a = 0, b = 0;
    for (uint32_t d = 0; d < la + lb; ++d) {
      split_at[ps + d] = a;
      const bool take_a = b == lb || (a < la && key[ps + a] < key[ps + la + b]);
      merged[ps + d] = take_a ? key[ps + a++] : key[ps + la + b++];
    }
    split_at[ps + la + lb] = la;   // the pair's end (the next pair's d = 0 is overwritten below)
  }
  for (uint64_t ps = 0; ps < n; ps += 2 * R) split_at[ps] = 0;
  const uint32_t ntiles = (n + P - 1) / P;
  const bool last_level = level + 1 == levels_for(n, T);
  uint64_t covered = 0;
  for (uint32_t j = 0; j < ntiles; ++j) {
    const sw::MergeTile m = sw::merge_tile(n, j, R, P);
    CHECK(m.ps % (2 * R) == 0 && m.o0 == (uint64_t)j * P && m.ps <= m.o0, "tile %u: pair start", j);
    const uint32_t la = (uint32_t)std::min<uint64_t>(R, n - m.ps), lb = (uint32_t)std::min<uint64_t>(R, n - m.ps - la);
    CHECK(m.la == la && m.lb == lb && m.d0 == m.o0 - m.ps && m.d1 == std::min(m.d0 + P, la + lb),
          "n=%u T=%u P=%u level=%u tile %u: geometry", n, T, P, level, j);
    CHECK(m.o0 == covered, "tile %u starts at %llu, the previous ended at %llu", j, (unsigned long long)m.o0,
          (unsigned long long)covered);
    covered += m.d1 - m.d0;
    const uint32_t s0 = split_at[m.ps + m.d0];
    // the next tile's own first split: in this pair when this tile does not
    // end the pair, otherwise any value (the next pair's, the next segment's,
    // or a slot nobody wrote)
    const bool ends_pair = m.d1 == la + lb;
    const uint32_t end_split = ends_pair ? (uint32_t)rng() : split_at[m.ps + m.d1];
    const sw::TileIO io = sw::tile_io(sw::TileRec{base, n, j, s0}, end_split, R, P, T, (int)level);
    const uint32_t a1 = ends_pair ? la : split_at[m.ps + m.d1];
    CHECK(io.na == (int)(a1 - s0) && io.cnt == (int)(m.d1 - m.d0), "n=%u T=%u P=%u level=%u tile %u: counts clamp",
          n, T, P, level, j);
    CHECK(io.ob == (size_t)base + m.o0, "tile %u: output position", j);
    const size_t a_lo = (size_t)base + m.ps, b_lo = a_lo + la;
    CHECK(io.apos >= a_lo && io.apos + io.na <= a_lo + la, "tile %u: A reads leave run A", j);
    CHECK(io.bpos >= b_lo && io.bpos + (io.cnt - io.na) <= b_lo + lb, "tile %u: B reads leave run B", j);
    // its inputs merged are the outputs it owns
    std::vector<uint32_t> in;
    for (int i = 0; i < io.na; ++i) in.push_back(key[io.apos - base + i]);
    for (int i = 0; i < io.cnt - io.na; ++i) in.push_back(key[io.bpos - base + i]);
    std::sort(in.begin(), in.end());
    CHECK(std::equal(in.begin(), in.end(), merged.begin() + (long)m.o0), "n=%u T=%u P=%u level=%u tile %u: inputs",
          n, T, P, level, j);
    CHECK((io.final != 0) == last_level, "tile %u: final flag", j);
  }
  CHECK(covered == n, "tiles cover %llu of %u", (unsigned long long)covered, n);
}

// 2. k_merge's range bookkeeping, with tile t's "split" being t itself
static void check_ranges(uint32_t ntiles, uint32_t G, uint32_t NG) {
  const uint32_t TB = NG - 1;
  std::vector<uint32_t> rec(TB), spl(TB + 1);
  const uint32_t q = ntiles / G, rem = ntiles % G;
  uint32_t next_tile = 0;
  for (uint32_t blk = 0; blk < G; ++blk) {
    const uint32_t nb = q + (blk < rem ? 1u : 0u);
    if (nb == 0) continue;
    const uint32_t tb = blk * q + std::min(blk, rem);
    CHECK(tb == next_tile, "block %u starts at tile %u, expected %u", blk, tb, next_tile);
    next_tile = tb + nb;
    std::fill(rec.begin(), rec.end(), ~0u);
    std::fill(spl.begin(), spl.end(), ~0u);
    auto place = [&](uint32_t t0) {
      for (uint32_t g = 0; g < NG; ++g) {
        if (!sw::place_group_active(t0, g, ntiles, tb + nb)) continue;
        spl[g] = t0 + g;
        if (g + 1 < NG) rec[g] = t0 + g;
      }
    };
    place(tb);
    uint32_t cur = rec[0], cur_end = spl[1];
    for (uint32_t k = 0; k < nb; ++k) {
      CHECK(cur == tb + k, "block %u tile %u: record of tile %u", blk, tb + k, cur);
      // the split of the tile after it (none after the class's last tile:
      // that tile ends its segment, so its end split is never read)
      CHECK(tb + k + 1 == ntiles || cur_end == tb + k + 1, "block %u tile %u: end split of tile %u", blk, tb + k,
            cur_end);
      const bool has_next = k + 1 < nb;
      const uint32_t kn = sw::place_slot(k + 1, TB);
      if (has_next && kn == 0) place(tb + k + 1);
      if (has_next) {
        cur = rec[kn];
        cur_end = spl[kn + 1];
      }
    }
  }
  CHECK(next_tile == ntiles, "ranges cover %u of %u tiles", next_tile, ntiles);
}

// 3. the K-ary search against upper_bound
static void check_search(std::mt19937_64& rng, uint32_t K) {
  for (int rep = 0; rep < 300; ++rep) {
    const uint32_t cact = 1 + (uint32_t)(rng() % (rep < 100 ? 20 : 5000));
    std::vector<uint32_t> mt(cact + 1, 0);
    for (uint32_t k = 1; k <= cact; ++k) mt[k] = mt[k - 1] + 1 + (uint32_t)(rng() % (rng() % 4 ? 3 : 400));
    int max_rounds = 0;
    for (uint32_t t = 0; t < mt[cact]; t += 1 + (uint32_t)(rng() % 7)) {
      sw::KarySearch ks{0, cact};
      int rounds = 0;
      while (ks.open()) {
        uint32_t c = 0;
        for (uint32_t gl = 0; gl < K; ++gl) {
          const uint32_t k = ks.probe(gl, K);
          c += (k < ks.hi && mt[k] <= t) ? 1u : 0u;
        }
        CHECK(c >= 1, "K=%u: no probe at or below tile %u", K, t);
        ks.narrow(c, K);
        ++rounds;
      }
      const uint32_t want = (uint32_t)(std::upper_bound(mt.begin(), mt.begin() + cact, t) - mt.begin()) - 1;
      CHECK(ks.lo == want, "K=%u cact=%u tile %u: segment %u, expected %u", K, cact, t, ks.lo, want);
      max_rounds = std::max(max_rounds, rounds);
    }
    int bound = 0;
    for (uint64_t span = 1; span < cact; span *= K) ++bound;
    CHECK(max_rounds <= bound + 1, "K=%u cact=%u: %d rounds", K, cact, max_rounds);
  }
}

int main() {
  std::mt19937_64 rng(1411);
  // 1. chosen edges, then random segments
  const uint32_t Ts[] = {16, 128, 1024, 2048, 8192};
  int cases = 0;
  for (uint32_t T : Ts)
    for (uint32_t P = 64; P <= 2 * T && P <= 4096; P *= 4)
      for (uint32_t n : {T + 1, 2 * T, 2 * T + 1, 3 * T, 4 * T - 1, 4 * T, 5 * T + P - 1, 7 * T + 3})
        for (uint32_t l = 0; l < levels_for(n, T); ++l, ++cases) check_level(rng, n, T, P, l);
  for (int rep = 0; rep < 44; ++rep) {
    const uint32_t T = Ts[rng() % 5];
    uint32_t P = 64u << (rng() % 7);
    while (P > 2 * T) P >>= 1;
    const uint32_t n = T + 1 + (uint32_t)(rng() % (rep < 40 ? 40 * T : (1u << 20)));
    for (uint32_t l = 0; l < levels_for(n, T); ++l, ++cases) check_level(rng, n, T, P, l);
  }
  // 2. ranges over grids of every size, for every group count a workgroup may have
  for (uint32_t NG : {16u, 32u, 64u, 128u})
    for (uint32_t ntiles : {1u, 2u, 15u, 16u, 17u, 100u, 1000u, 4097u})
      for (uint32_t G : {1u, 2u, 3u, 7u, 64u, 256u, 1024u, 5000u}) check_ranges(ntiles, G, NG);
  // 3. the segment search with groups of 2..16 lanes
  for (uint32_t K : {2u, 4u, 8u, 16u}) check_search(rng, K);
  std::printf("tile levels checked: %d\nOK\n", cases);
  return 0;
}
