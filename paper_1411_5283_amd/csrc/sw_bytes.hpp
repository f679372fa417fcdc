// sw_bytes.hpp -- byte-level helpers of the text kernels as plain integer
// code, also built for the host by their tests: the tokenizer's byte classes
// as bit masks, four bytes at a time (a letter is an ASCII letter;
// whitespace is tab, line feed, vertical tab, form feed, carriage return or
// space; every other byte is special), and the stores that write a word's
// text from its key lanes a dword at a time.
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

// A word's text from its key lanes: its L bytes (big-endian lanes ln[0..3],
// byte j at bits 63-8(j%8) of lane j/8; whatever the lanes hold past the
// word is masked off), then the separator when sw = 1.  The word starts at
// byte o (0..3) of the aligned destination dst; output dword k covers word
// bytes 4k-o .. 4k-o+3, built from two consecutive dwords of the word with
// one funnel shift.  Dwords wholly inside the word are stored whole, the
// word's first and last dwords (shared with its neighbours) byte- and
// halfword-wise, so that words written by different threads never overlap.
__host__ __device__ inline void store_part(uint8_t* dst, uint32_t v, uint32_t fb, uint32_t lb) {
  // bytes [fb, lb) of v to dst[fb..lb): a byte to reach an even address, then
  // a halfword, then a last byte
  uint32_t p = fb;
  if ((p & 1u) && p < lb) {
    dst[p] = (uint8_t)(v >> (8 * p));
    ++p;
  }
  if (p + 2 <= lb) {
    *(uint16_t*)(dst + p) = (uint16_t)(v >> (8 * p));
    p += 2;
  }
  if (p < lb) dst[p] = (uint8_t)(v >> (8 * p));
}

template <class P>
__host__ __device__ inline void put_word_text(P dst, uint32_t o, const uint64_t (&ln)[4], uint32_t L, uint32_t sw,
                                              uint32_t sep) {
  const uint32_t n = L + sw;
  if (n == 0) return;
  const uint32_t K = (o + n - 1) >> 2;           // last output dword
  const uint32_t last = ((o + n - 1) & 3u) + 1;  // bytes of it that are the word's
  const uint32_t ks = (o + L) >> 2, sepv = (sep & 255u) << (8 * ((o + L) & 3u));
  uint32_t W[9];   // word bytes 4i..4i+3, little-endian
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    W[2 * i] = __builtin_bswap32((uint32_t)(ln[i] >> 32));
    W[2 * i + 1] = __builtin_bswap32((uint32_t)ln[i]);
  }
  W[8] = 0;
#pragma unroll
  for (uint32_t k = 0; k < 9; ++k) {
    if (k <= K) {
      const uint64_t two = ((uint64_t)W[k] << 32) | (k ? W[k - 1] : 0u);
      uint32_t v = (uint32_t)(two >> (32 - 8 * o));
      const int keep = (int)(L + o) - 4 * (int)k;   // output bytes of this dword below the word's end
      v &= keep >= 4 ? ~0u : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
      if (sw && k == ks) v |= sepv;
      const uint32_t fb = k == 0 ? o : 0u, lb = k == K ? last : 4u;
      if (fb == 0 && lb == 4)
        *(uint32_t*)(dst + 4 * k) = v;
      else
        store_part((uint8_t*)(dst + 4 * k), v, fb, lb);
    }
  }
}

}  // namespace sw
