// The dword-at-a-time writer of a word's text from its key lanes
// (csrc/sw_bytes.hpp, the code the sorted-text kernel uses), checked on the
// host against the text written byte by byte: every length 0..32, every
// start within a dword, with and without a separator, lanes holding garbage
// past the word; then runs of random words written back to back in random
// order, where each word's edge dwords are shared with its neighbours.
#define __host__
#define __device__
#include "sw_bytes.hpp"

#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

static void lanes_of(const uint8_t* w, uint32_t L, uint64_t garbage, uint64_t (&ln)[4]) {
  for (int q = 0; q < 4; ++q) {
    uint64_t v = 0;
    for (int b = 0; b < 8; ++b) {
      const uint32_t j = 8 * q + b;
      const uint64_t byte = j < L ? w[j] : ((garbage >> (8 * (j % 8))) & 255u);
      v |= byte << (56 - 8 * b);
    }
    ln[q] = v;
  }
}

int main() {
  std::mt19937_64 rng(14115283);
  const uint32_t seps[] = {10u, 0u, 255u, 32u};
  for (uint32_t L = 0; L <= 32; ++L) {
    for (uint32_t sw = 0; sw < 2; ++sw) {
      for (uint32_t o = 0; o < 4; ++o) {
        for (int rep = 0; rep < 200; ++rep) {
          uint8_t w[32];
          for (auto& b : w) b = (uint8_t)rng();
          uint64_t ln[4];
          lanes_of(w, L, rep % 2 ? rng() : 0ull, ln);
          const uint32_t sep = seps[rep % 4];
          uint32_t buf32[12];
          uint8_t* buf = (uint8_t*)buf32;
          std::memset(buf, 0xAB, sizeof(buf32));
          sw::put_word_text(buf, o, ln, L, sw, sep);
          uint8_t want[48];
          std::memset(want, 0xAB, sizeof(want));
          std::memcpy(want + o, w, L);
          if (sw) want[o + L] = (uint8_t)sep;
          if (std::memcmp(buf, want, sizeof(want)) != 0) {
            std::printf("mismatch: L=%u sw=%u o=%u rep=%d\n", L, sw, o, rep);
            return 1;
          }
        }
      }
    }
  }
  for (int it = 0; it < 2000; ++it) {
    const int nw = 1 + (int)(rng() % 300);
    const uint32_t sw = (uint32_t)(rng() % 2), sep = (uint32_t)(rng() % 256);
    const uint32_t lmax = 1 + (uint32_t)(rng() % 32);
    std::vector<std::vector<uint8_t>> words(nw);
    std::vector<uint32_t> at(nw);
    const uint32_t start = (uint32_t)(rng() % 4);
    uint32_t pos = start;
    for (int i = 0; i < nw; ++i) {
      words[i].resize(rng() % (lmax + 1));
      for (auto& b : words[i]) b = (uint8_t)rng();
      at[i] = pos;
      pos += (uint32_t)words[i].size() + sw;
    }
    std::vector<uint32_t> buf32(pos / 4 + 2, 0xABABABABu);
    uint8_t* buf = (uint8_t*)buf32.data();
    std::vector<int> order(nw);
    for (int i = 0; i < nw; ++i) order[i] = i;
    for (int i = nw - 1; i > 0; --i) std::swap(order[i], order[rng() % (i + 1)]);
    for (int i : order) {
      uint64_t ln[4];
      const uint32_t L = (uint32_t)words[i].size();
      lanes_of(words[i].data(), L, rng(), ln);
      sw::put_word_text(buf + (at[i] & ~3u), at[i] & 3u, ln, L, sw, sep);
    }
    std::vector<uint8_t> want(buf32.size() * 4, 0xAB);
    for (int i = 0; i < nw; ++i) {
      if (!words[i].empty()) std::memcpy(&want[at[i]], words[i].data(), words[i].size());
      if (sw) want[at[i] + words[i].size()] = (uint8_t)sep;
    }
    if (std::memcmp(buf, want.data(), want.size()) != 0) {
      std::printf("run mismatch: it=%d words=%d sw=%u start=%u\n", it, nw, sw, start);
      return 1;
    }
  }
  std::printf("OK\n");
  return 0;
}
