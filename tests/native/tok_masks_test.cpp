// The tokenizer's four-bytes-at-a-time byte classes and word-start addition
// (csrc/sw_bytes.hpp, the code the GPU kernels use), checked on the host
// against the reading applied byte by byte: every byte value in every lane
// of a dword next to several neighbours, and random 64-byte chunks (letters,
// whitespace, specials, bytes above 127, a ragged end of zero bytes) under
// each incoming state.
#define __host__
#define __device__
#include "sw_bytes.hpp"

#include <cstdio>
#include <random>

static bool is_space(uint32_t c) { return c == 32u || (c >= 9u && c <= 13u); }
static bool is_letter(uint32_t c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

int main() {
  const uint32_t neighbours[] = {0x00u, 0x20u, 0x41u, 0x7Au, 0x80u, 0xFFu, 0x09u, 0x2Du};
  for (uint32_t c = 0; c < 256; ++c) {
    for (int pos = 0; pos < 4; ++pos) {
      for (uint32_t nb : neighbours) {
        uint32_t w = 0;
        for (int t = 0; t < 4; ++t) w |= (t == pos ? c : nb) << (8 * t);
        const uint32_t L = sw::swar_pack4(sw::swar_letters(w)), S = sw::swar_pack4(sw::swar_spaces(w));
        for (int t = 0; t < 4; ++t) {
          const uint32_t b = (w >> (8 * t)) & 255u;
          if (((L >> t) & 1u) != (uint32_t)is_letter(b) || ((S >> t) & 1u) != (uint32_t)is_space(b)) {
            std::printf("byte class mismatch: byte %u in lane %d next to %u\n", c, pos, nb);
            return 1;
          }
        }
      }
    }
  }
  std::mt19937_64 rng(14115283);
  const char alphabet[] = "abcxyzABCXYZ \t\n\r\v\f-'.,09@[`{";
  const int na = (int)sizeof(alphabet) - 1;
  for (int it = 0; it < 200000; ++it) {
    uint8_t buf[64];
    const int n = (int)(rng() % 65);
    for (int i = 0; i < 64; ++i) buf[i] = i < n ? (rng() % 4 ? (uint8_t)alphabet[rng() % na] : (uint8_t)rng()) : 0;
    uint32_t w[16];
    for (int j = 0; j < 16; ++j)
      w[j] = buf[4 * j] | buf[4 * j + 1] << 8 | buf[4 * j + 2] << 16 | (uint32_t)buf[4 * j + 3] << 24;
    const sw::TokMasks m = sw::tok_masks(w);
    for (int in = 0; in < 3; ++in) {   // incoming state: none, whitespace, letter
      uint64_t want = 0, letters = 0, spaces = 0;
      int cur = in;
      for (int i = 0; i < 64; ++i) {
        if (is_space(buf[i])) {
          spaces |= 1ull << i;
          cur = 1;
        } else if (is_letter(buf[i])) {
          letters |= 1ull << i;
          if (cur != 2) want |= 1ull << i;
          cur = 2;
        }
      }
      const uint64_t got = sw::tok_starts(m, in != 2);
      if (m.letter != letters || m.space != spaces || got != want) {
        std::printf("chunk %d, incoming state %d: starts %llx, expected %llx\n", it, in,
                    (unsigned long long)got, (unsigned long long)want);
        return 1;
      }
    }
  }
  std::printf("OK\n");
  return 0;
}
