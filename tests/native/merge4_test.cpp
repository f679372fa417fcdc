// The streamed four-way merge level (csrc/sw_merge4.hpp, the phases the
// merge kernel runs between barriers) driven on the host thread by thread,
// with the kernel's walk over workgroup ranges, segments and groups and the
// split search for groups entered in the middle.  Checked against a plain
// sort of each group: segments of many sizes (groups of one to four runs,
// short last runs), several workgroup counts (ranges starting anywhere),
// small and full-size step and ring geometries, one-lane and two-lane keys,
// and LDS full of random keys at the start of every piece (so no output may
// lean on a slot that holds no real item or end marker).  Prints "OK" and exits 0, or
// names the failing case and exits 1.
#define __host__
#define __device__
#include "sw_merge4.hpp"

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

using namespace sw;

// A key buffer on the host (structure of arrays, as in HBM).
struct HostBuf {
  std::vector<uint64_t> k[4];
  std::vector<uint32_t> idx;
  KeyBuf view() {
    KeyBuf b;
    for (int q = 0; q < 4; ++q) b.k[q] = k[q].data();
    b.idx = idx.data();
    return b;
  }
  void resize(size_t n) {
    for (int q = 0; q < 4; ++q) k[q].assign(n, 0);
    idx.assign(n, 0);
  }
};

template <int NL>
static Key<NL> make_key(uint64_t v, uint32_t i) {
  Key<NL> k;
  if constexpr (NL == 0) {
    k.k = (v << 32) | i;   // class 0: four key bytes above the index
  } else {
    for (int q = 0; q < NL; ++q) k.k[q] = q == NL - 1 ? v : 0x6162636465666768ull;
    k.idx = i;
  }
  return k;
}

// Co-ranks by the split search, slot by slot (the kernel's rounds).
template <class M, int NL>
static void split_host(typename M::Lds& L, const KeyBuf& src, const uint64_t (&st)[4], const uint32_t (&len)[4],
                       uint32_t d, uint32_t (&sp)[4]) {
  SplitScratch<Key<NL>>& S = L.u.sp;
  split_init(S, len, d);
  while (!S.done) {
    CHECK(S.rounds < (uint32_t)kSplitMaxRounds, "split did not close");
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < kSplitSlots; ++j) {
        const uint32_t p = split_slot_pos(S, i, j);
        S.pos[i][j] = p;
        if (p != kSplitNone) {
          CHECK(p < len[i], "split reads past a run");
          S.key[i][j] = gload<NL>(src, (size_t)(st[i] + p));
        }
      }
    split_begin_round(S);
    for (int i = 0; i < 4; ++i)
      for (int j = 1; j + 1 < kSplitSlots; ++j) {
        if (S.pos[i][j] == kSplitNone) continue;
        const int v = split_decide(S, i, j, typename M::Less());
        if (v < 0) S.newlo[i] = std::max(S.newlo[i], S.pos[i][j] + 1);
        if (v > 0) S.newhi[i] = std::min(S.newhi[i], S.pos[i][j]);
      }
    split_finish_round(S);
  }
  uint32_t sum = 0;
  for (int i = 0; i < 4; ++i) sum += (sp[i] = S.lo[i]);
  CHECK(sum == d, "split sums to %u, not %u", sum, d);
}

// LDS as a fresh workgroup might find it: every slot of the rings and of X
// and Y holds a random key (smaller or larger than real ones), so an output
// that leaned on a slot it should not read would come out wrong.
template <class Lds, int NL>
static void poison_lds(Lds& L, std::mt19937_64& rng) {
  uint64_t* p = reinterpret_cast<uint64_t*>(&L.ring[0]);
  const size_t words = (sizeof(L.ring) + sizeof(L.u)) / sizeof(uint64_t);
  for (size_t i = 0; i < words; ++i) p[i] = rng();
}

// One level of the kernel: G workgroups, segments back to back (wp = their
// prefix), every phase run thread by thread.
template <int NL, int NT, int E, int PS, int RC>
static void run_level(const KeyBuf& src, const KeyBuf& dst, const std::vector<uint32_t>& wp, uint64_t R, uint32_t G) {
  using M = M4<NL, NT, E, PS, RC>;
  using K = Key<NL>;
  constexpr int FE = M::FE;
  static typename M::Lds L;
  static std::mt19937_64 rng_poison(77);
  auto poison = [](typename M::Lds& l, std::mt19937_64& g) { poison_lds<typename M::Lds, NL>(l, g); };
  // the seals as the threads run them: each thread updates the state, thread
  // r (x) writes run r's (side x's) sentinel; here one copy of the state
  auto seal_runs_all = [](typename M::Lds& l, typename M::State& st) {
    typename M::State probe = st;
    for (uint32_t t = 0; t < 4; ++t) {
      probe = st;
      M::seal_runs(l, probe, t);
    }
    st = probe;
  };
  auto seal_xy_all = [](typename M::Lds& l, typename M::State& st, uint32_t a, uint32_t b) {
    typename M::State probe = st;
    for (uint32_t t = 0; t < 2; ++t) {
      probe = st;
      M::seal_xy(l, probe, t, a, b);
    }
    st = probe;
  };
  const uint32_t nseg = (uint32_t)wp.size() - 1;
  const uint64_t total = wp[nseg];
  for (uint32_t b = 0; b < G; ++b) {
    const uint64_t r0 = total * b / G, r1 = total * (b + 1) / G;
    if (r0 >= r1) continue;
    uint32_t k = (uint32_t)(std::upper_bound(wp.begin(), wp.begin() + nseg, (uint32_t)r0) - wp.begin()) - 1;
    for (uint64_t pos = r0; pos < r1;) {
      while (wp[k + 1] <= pos) ++k;
      const uint32_t base = wp[k], n = wp[k + 1] - wp[k];
      const M4Group g = m4_group(n, pos - base, R);
      const uint64_t gend = base + g.start + g.size;
      const uint32_t count = (uint32_t)(std::min<uint64_t>(gend, r1) - pos);
      const size_t ob = (size_t)base + g.start + g.d;
      uint64_t st[4];
      for (int r = 0; r < 4; ++r) st[r] = (uint64_t)base + g.start + g.run_off[r];
      uint32_t sp[4] = {0, 0, 0, 0};
      if (g.d > 0) split_host<M, NL>(L, src, st, g.len, g.d, sp);
      typename M::State s;
      M::begin(s, st, g.len, sp);
      poison(L, rng_poison);
      M::fill_amounts(s, 4u * RC);
      for (uint32_t q = 0; q < M::refill_total(s); ++q) {
        K v;
        if (M::refill_load(s, src, q, v)) M::refill_put(L, s, q, v);
      }
      L.end[0][0] = L.end[0][1] = L.end[1][0] = L.end[1][1] = 0;
      M::refill_done(s);
      seal_runs_all(L, s);
      uint32_t wx = M::want(s, 0), wy = M::want(s, 1);
      for (uint32_t wi = 0; wi < M::topup_items(s); ++wi) M::topup(L, s, wi);
      seal_xy_all(L, s, wx, wy);
      M::topup_done(s, L, wx, wy);
      M::fill_amounts(s, 4u * RC);
      for (uint32_t q = 0; q < M::refill_total(s); ++q) {
        K v;
        if (M::refill_load(s, src, q, v)) M::refill_put(L, s, q, v);
      }
      M::refill_done(s);
      seal_runs_all(L, s);
      static K pf[NT][FE];
      for (uint32_t done = 0; done < count;) {
        for (uint32_t t = 0; t < (uint32_t)NT; ++t)
          for (int u = 0; u < FE; ++u) {
            const uint32_t q = t + (uint32_t)u * NT;
            if (q < M::refill_total(s)) M::refill_put(L, s, q, pf[t][u]);
          }
        M::refill_done(s);
        seal_runs_all(L, s);
        CHECK(!M::fill_amounts(s, (uint32_t)(FE * NT)), "in-flight loads exceed the registers");
        for (int r = 0; r < 4; ++r)
          CHECK(s.valid[r] + s.fly[r] <= (uint32_t)RC, "ring %d overfull", r);
        for (uint32_t t = 0; t < (uint32_t)NT; ++t)
          for (int u = 0; u < FE; ++u) M::refill_load(s, src, t + (uint32_t)u * NT, pf[t][u]);
        L.end[0][0] = L.end[0][1] = L.end[1][0] = L.end[1][1] = 0;
        // B: every run not at its end holds at least PS items; a run at its
        // end with fewer than PS items has its sentinel in place
        for (int r = 0; r < 4; ++r) {
          const bool at_end = s.cons[r] + s.valid[r] == s.len[r];
          CHECK(at_end || s.valid[r] >= (uint32_t)PS, "run %d starved: %u items", r, s.valid[r]);
          CHECK(!at_end || s.valid[r] >= (uint32_t)PS || (s.sealed & (1u << r)), "run %d end unmarked", r);
        }
        wx = M::want(s, 0);
        wy = M::want(s, 1);
        for (uint32_t wi = 0; wi < M::topup_items(s); ++wi) M::topup(L, s, wi);
        seal_xy_all(L, s, wx, wy);
        M::topup_done(s, L, wx, wy);
        for (int x = 0; x < 2; ++x) {
          const bool ended = s.cons[2 * x] == s.len[2 * x] && s.cons[2 * x + 1] == s.len[2 * x + 1];
          CHECK(ended || s.px[x] - s.cx[x] == (uint32_t)PS, "side %d holds %u items", x, s.px[x] - s.cx[x]);
          CHECK(!ended || s.px[x] - s.cx[x] == (uint32_t)PS || (s.sealed & (16u << x)), "side %d end unmarked", x);
        }
        const uint32_t cnt = std::min<uint32_t>(count - done, PS);
        static K out[NT][E];
        static uint32_t nout[NT];
        for (uint32_t t = 0; t < (uint32_t)NT; ++t) nout[t] = M::final_merge(L, s, t, cnt, out[t]);
        M::final_done(s, L, cnt);
        uint32_t stored = 0;
        for (uint32_t t = 0; t < (uint32_t)NT; ++t) {
          const size_t o = ob + done + (size_t)t * E;
          for (uint32_t j = 0; j < nout[t]; ++j) gstore<NL>(dst, o + j, out[t][j]);
          stored += nout[t];
        }
        CHECK(stored == cnt, "step stored %u of %u", stored, cnt);
        done += cnt;
      }
      pos += count;
    }
  }
}

template <int NL, int NT, int E, int PS, int RC>
static void check_level(std::mt19937_64& rng, const std::vector<uint32_t>& sizes, uint64_t R, uint32_t G, int keymode) {
  std::vector<uint32_t> wp(1, 0);
  for (uint32_t n : sizes) wp.push_back(wp.back() + n);
  const uint32_t N = wp.back();
  HostBuf a, b;
  a.resize(N + 1);
  b.resize(N + 1);
  KeyBuf src = a.view(), dst = b.view();
  std::vector<std::vector<Key<NL>>> want(sizes.size());
  for (size_t k = 0; k < sizes.size(); ++k) {
    const uint32_t n = sizes[k];
    std::vector<Key<NL>> keys(n);
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t v = keymode == 0 ? rng() % 1000003 : (keymode == 1 ? rng() % 5 : (uint64_t)(i / 37));
      keys[i] = make_key<NL>(v & 0xFFFFFFFFull, i);
    }
    // runs of R sorted in place: the input of a level
    for (uint32_t r0 = 0; r0 < n; r0 += (uint32_t)R) {
      auto e = keys.begin() + std::min<uint64_t>(n, r0 + R);
      std::sort(keys.begin() + r0, e, typename M4<NL, NT, E, PS, RC>::Less());
    }
    for (uint32_t i = 0; i < n; ++i) gstore<NL>(src, wp[k] + i, keys[i]);
    // expected: every group of four runs sorted
    want[k] = keys;
    for (uint64_t g0 = 0; g0 < n; g0 += 4 * R) {
      auto e = want[k].begin() + std::min<uint64_t>(n, g0 + 4 * R);
      std::sort(want[k].begin() + g0, e, typename M4<NL, NT, E, PS, RC>::Less());
    }
  }
  run_level<NL, NT, E, PS, RC>(src, dst, wp, R, G);
  for (size_t k = 0; k < sizes.size(); ++k)
    for (uint32_t i = 0; i < sizes[k]; ++i) {
      const Key<NL> got = gload<NL>(dst, wp[k] + i);
      const Key<NL>& exp = want[k][i];
      const typename M4<NL, NT, E, PS, RC>::Less less;
      CHECK(!less(got, exp) && !less(exp, got), "NL=%d PS=%d RC=%d R=%llu G=%u segment %zu (n=%u) position %u differs",
            NL, PS, RC, (unsigned long long)R, G, k, sizes[k], i);
    }
}

int main() {
  std::mt19937_64 rng(5283);
  // segment sizes: one run, part of a run, 2-4 runs, several groups, short tails
  const std::vector<std::vector<uint32_t>> shapes = {
      {1}, {7}, {16}, {17}, {33, 64, 65}, {200, 3, 511, 1000}, {4096}, {4097, 1, 2500}, {10000}};
  for (const auto& sz : shapes)
    for (uint32_t G : {1u, 3u, 7u, 64u})
      for (int km = 0; km < 3; ++km) {
        check_level<0, 4, 2, 8, 16>(rng, sz, 16, G, km);       // R = 16: groups of 64
        check_level<0, 8, 4, 32, 64>(rng, sz, 40, G, km);      // R not a power of two
        check_level<2, 4, 4, 16, 32>(rng, sz, 64, G, km);      // two-lane keys
        check_level<1, 8, 2, 16, 64>(rng, sz, 8, G, km);       // rings four steps deep
      }
  // full-size geometry of the kernel, larger segments, higher levels
  for (int t = 0; t < 6; ++t) {
    std::vector<uint32_t> sz;
    for (int k = 0; k < 3; ++k) sz.push_back(1000 + (uint32_t)(rng() % 200000));
    const uint64_t R = 2048ull << (2 * (t % 3));
    for (uint32_t G : {5u, 200u}) {
      check_level<0, 256, 2, 512, 1024>(rng, sz, R, G, t % 3);
      check_level<1, 128, 2, 256, 512>(rng, sz, R, G, (t + 1) % 3);
    }
  }
  std::printf("OK\n");
  return 0;
}
