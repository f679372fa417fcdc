// sw_keys.hpp -- keys of the gfx950 word sort and their HBM buffers, as plain
// code built for the device and, by the merge tests, for the host.
//
// A word of length L is packed into big-endian 64-bit lanes, zero padded;
// for two words of the same length, comparing the lanes as unsigned
// integers, most significant lane first, is the same as comparing the bytes.
// The original index breaks ties, so every key is distinct.  Class 0 (L <= 4)
// packs its four key bytes and the index into one u64.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace sw {

// Structure-of-arrays key buffer in HBM: lanes k[0..3] and the index.
struct KeyBuf {
  uint64_t* k[4];
  uint32_t* idx;
};

// ---------------------------------------------------------------- keys
template <int NL>
struct Key {
  uint64_t k[NL];
  uint32_t idx;
};
template <>
struct Key<0> {
  uint64_t k;
};

// Lexicographic: lane 0 first, then the index.  Written with bitwise
// and/or of the comparisons so that on the GPU they combine as wave masks
// (scalar instructions), not as selects of 0/1 values.
template <int NL>
__host__ __device__ inline bool key_less(const Key<NL>& a, const Key<NL>& b) {
  bool lt = a.idx < b.idx;
#pragma unroll
  for (int q = NL - 1; q >= 0; --q) lt = (a.k[q] < b.k[q]) | ((a.k[q] == b.k[q]) & lt);
  return lt;
}
template <>
__host__ __device__ inline bool key_less<0>(const Key<0>& a, const Key<0>& b) {
  return a.k < b.k;
}

template <int NL>
__host__ __device__ inline Key<NL> key_sentinel() {
  Key<NL> s;
#pragma unroll
  for (int q = 0; q < NL; ++q) s.k[q] = ~0ull;
  s.idx = ~0u;
  return s;
}
template <>
__host__ __device__ inline Key<0> key_sentinel<0>() {
  Key<0> s;
  s.k = ~0ull;
  return s;
}

// The fill of a tile's slots past its last real item: one below the
// sentinel, so above every real key (a workspace holds at most 2^32 - 2
// words, so a real index is at most 2^32 - 3).  The LDS merge rounds rely on
// every item of a run lying strictly below the sentinel slot that ends it.
template <int NL>
__host__ __device__ inline Key<NL> key_fill() {
  Key<NL> s = key_sentinel<NL>();
  s.idx = ~0u - 1u;
  return s;
}
template <>
__host__ __device__ inline Key<0> key_fill<0>() {
  Key<0> s;
  s.k = ~0ull - 1ull;
  return s;
}

template <int NL>
__host__ __device__ inline uint32_t key_index(const Key<NL>& v) { return v.idx; }
template <>
__host__ __device__ inline uint32_t key_index<0>(const Key<0>& v) { return (uint32_t)v.k; }

template <int NL>
__host__ __device__ inline Key<NL> gload(const KeyBuf& b, size_t p) {
  Key<NL> v;
#pragma unroll
  for (int q = 0; q < NL; ++q) v.k[q] = b.k[q][p];
  v.idx = b.idx[p];
  return v;
}
template <>
__host__ __device__ inline Key<0> gload<0>(const KeyBuf& b, size_t p) {
  Key<0> v;
  v.k = b.k[0][p];
  return v;
}

template <int NL>
__host__ __device__ inline void gstore(const KeyBuf& b, size_t p, const Key<NL>& v) {
#pragma unroll
  for (int q = 0; q < NL; ++q) b.k[q][p] = v.k[q];
  b.idx[p] = v.idx;
}
template <>
__host__ __device__ inline void gstore<0>(const KeyBuf& b, size_t p, const Key<0>& v) {
  b.k[0][p] = v.k;
}

template <int NL>
__host__ __device__ inline Key<NL> key_select(bool c, const Key<NL>& x, const Key<NL>& y) {
  Key<NL> r;
#pragma unroll
  for (int q = 0; q < NL; ++q) r.k[q] = c ? x.k[q] : y.k[q];
  r.idx = c ? x.idx : y.idx;
  return r;
}
template <>
__host__ __device__ inline Key<0> key_select<0>(bool c, const Key<0>& x, const Key<0>& y) {
  Key<0> r;
  r.k = c ? x.k : y.k;
  return r;
}

}  // namespace sw
