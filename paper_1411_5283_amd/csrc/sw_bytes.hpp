// sw_bytes.hpp -- the tokenizer's byte classes as bit masks, four bytes at
// a time (plain integer code, also built for the host by its test).  A
// letter is an ASCII letter; whitespace is tab, line feed, vertical tab, form
// feed, carriage return or space; every other byte is special.
#pragma once

#include <cstdint>

namespace sw {

// Four bytes at a time: bit 7 of each byte of the result flags a letter
// (resp. whitespace).  Every byte is brought below 128 before adding, so no
// sum carries into the next byte; bytes of 128 and above are neither.
__host__ __device__ inline uint32_t swar_letters(uint32_t w) {
  const uint32_t x = (w | 0x20202020u) & 0x7F7F7F7Fu;   // case folded
  const uint32_t ge_a = x + 0x1F1F1F1Fu;                 // bit 7: byte >= 'a'
  const uint32_t ge_brace = x + 0x05050505u;             // bit 7: byte >= '{'
  return ge_a & ~ge_brace & ~w & 0x80808080u;
}
__host__ __device__ inline uint32_t swar_spaces(uint32_t w) {
  const uint32_t y = w ^ 0x20202020u;                                      // zero where w is ' '
  const uint32_t eq = ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) & 0x80808080u;
  const uint32_t x = w & 0x7F7F7F7Fu;
  const uint32_t ge9 = x + 0x77777777u;                                    // bit 7: byte >= 9
  const uint32_t ge14 = x + 0x72727272u;                                   // bit 7: byte >= 14
  return eq | (ge9 & ~ge14 & ~w & 0x80808080u);
}
// bit 7 of each byte -> bits 0..3
__host__ __device__ inline uint32_t swar_pack4(uint32_t f) {
  f >>= 7;
  return (f | (f >> 7) | (f >> 14) | (f >> 21)) & 0xFu;
}

// The thread's 64 bytes as bit masks (bit i: byte i), letters and whitespace.
struct TokMasks {
  uint64_t letter, space;
};
__host__ __device__ inline TokMasks tok_masks(const uint32_t (&w)[16]) {
  TokMasks m{0, 0};
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    m.letter |= (uint64_t)swar_pack4(swar_letters(w[j])) << (4 * j);
    m.space |= (uint64_t)swar_pack4(swar_spaces(w[j])) << (4 * j);
  }
  return m;
}

// Word starts among the thread's bytes: a letter whose last non-special byte
// before it is whitespace (or, for the first one, the incoming state when
// `space_in`).  Adding 1 just above each space (and at bit 0 for space_in)
// to the mask of special bytes carries through the specials that follow and
// lands on the first non-special byte after them.
__host__ __device__ inline uint64_t tok_starts(const TokMasks& m, bool space_in) {
  const uint64_t special = ~(m.letter | m.space);
  return ((special + (m.space << 1) + (space_in ? 1ull : 0ull)) & ~special) & m.letter;
}

}  // namespace sw
