// sw_device.hpp -- device-side types and helpers of the gfx950 word sort.
//
// Key representation.  Words of one length L are compared as L bytes,
// unsigned, most significant first (the "alphabetic" order of section 3's
// phase 3, read as byte order).  A word is packed into big-endian 64-bit
// lanes, zero padded: for two words of the SAME length, comparing the lanes
// as unsigned integers, most significant lane first, is the same as
// comparing the bytes.  The original index breaks ties, which is the order
// bubble sort leaves equal words in, so every key is distinct and the sort
// has exactly one correct result.
//
// Key classes by length (fixed-width rows, the paper's 3-D char array):
//   class 0: L 0..4    one u64 = (4 key bytes << 32) | index
//   class 1: L 5..8    one lane + u32 index
//   class 2: L 9..16   two lanes + u32 index
//   class 3: L 17..24  three lanes + u32 index
//   class 4: L 25..32  four lanes + u32 index
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_keys.hpp"
#include "sw_tiles.hpp"

namespace sw {

constexpr int kMaxLen = 32;
constexpr int kNB = kMaxLen + 1;        // buckets L = 0..32
constexpr int kNOff = kMaxLen + 2;      // bucket offsets per document
constexpr int kNClass = 5;
constexpr int kMaxLev = 24;             // merge levels a segment may need
constexpr uint32_t kWordsPerBlock = 4096;
constexpr uint32_t kSegsPerBlock = 4096;
// Short segments (at most kPackMax words) are sorted several to a tile of
// kPackTile items by k_sort_packed.
constexpr uint32_t kPackTile = 2048;
constexpr uint32_t kPackMax = kPackTile / 2;
constexpr int kNKeys = kNClass * kMaxLev + 1;   // segment-order keys (+1: empty)
constexpr int kKeyBits = 7;
static_assert(kNKeys <= (1 << kKeyBits), "segment key bits");

// device status bits
enum : uint32_t { ST_INVALID = 1u, ST_TOO_LONG = 2u, ST_WORKSPACE = 4u };

__host__ __device__ inline int class_of_len(uint32_t L) {
  return L <= 4 ? 0 : (L <= 8 ? 1 : (L <= 16 ? 2 : (L <= 24 ? 3 : 4)));
}
// lanes stored per class (class 0 is packed with the index): the fewest
// 8-byte lanes that hold the class's longest word
__host__ __device__ constexpr int lanes_of_class(int c) { return c; }

// Merge levels a segment of n items needs when tiles of T items come out of
// the chunk sort already sorted: runs double each level until one run holds n.
__host__ __device__ inline uint32_t levels_for(uint32_t n, uint32_t T) {
  uint32_t m = 0;
  uint64_t r = T;
  while (r < n) {
    r <<= 1;
    ++m;
  }
  return m;
}

// HBM merge passes of such a segment when each pass merges `fan` runs (2 or
// 4) into one: a four-way pass does two doublings.
__host__ __device__ inline uint32_t merge_passes(uint32_t n, uint32_t T, uint32_t fan) {
  const uint32_t m = levels_for(n, T);
  return fan == 4 ? (m + 1) / 2 : m;
}


// ---------------------------------------------------------------- run state
struct RunDesc {
  const uint8_t* chars;
  const uint32_t* offsets;
  const uint32_t* doc_offsets;   // null: one document of n_words words
  uint32_t* out_perm;
  uint32_t* out_boff;
  uint32_t n_words;              // used when doc_offsets is null
  uint32_t n_docs;
  uint8_t* out_text;             // non-null: also write the sorted text
  int32_t sep;                   // its separator byte, or none when negative
};

struct Header {
  RunDesc d;
  uint32_t status;               // ST_* bits
  uint32_t abort;                // nonzero: later kernels do nothing
  uint32_t n_docs;               // documents in this run
  uint32_t n_words;
  uint32_t n_blocks;             // word blocks (never spanning documents)
  uint32_t n_segs;               // n_docs * kNB
  uint32_t n_segblocks;
  uint32_t cls_start[kNClass + 1];         // class sublists of the ordered segments
  uint32_t active[kNClass][kMaxLev];       // segments of a class with more levels than l
  uint32_t pack_start[kNClass];            // first short segment of each class sublist
  uint32_t sort_tiles[kNClass];
  uint32_t pack_words[kNClass];            // words in the short segments of each class
};


// Workspace view handed to every kernel (by value).
struct Ws {
  Header* h;
  uint32_t* doc_off;    // [Dmax+1]  word offset of each document
  uint32_t* doc_blk;    // [Dmax+1]  first word block of each document
  uint32_t* cnt;        // [kNB][Bmax+1]  per-block length counts, then their prefix
  uint32_t* seg_n;      // [Dmax*kNB]  words of (document, length)
  uint32_t* seg_base;   // [Dmax*kNB]  first output position of the segment
  uint32_t* segcnt;     // [kNKeys][SBmax+1]
  uint32_t* sorted;     // [Smax]      non-empty segments by (class, levels desc)
  uint32_t* st;         // [Smax+kNClass]  chunk-sort tile prefix per class
  uint32_t* mt;         // [Smax+kNClass]  merge tile prefix per class
  uint32_t* vpre;       // [Smax+kNClass]  prefix of short-segment sizes per class
  uint32_t* wpre;       // [Smax+kNClass]  word prefix of the other segments per class
  KeyBuf a;             // key buffer 0 (scatter output, chunk sort in place)
  KeyBuf b;             // key buffer 1 (ping-pong for merge levels)
  uint32_t Nmax, Dmax, Bmax, Smax, SBmax;
  uint64_t Cmax;            // characters a run may span (offsets[N] - offsets[0])
  uint32_t T[kNClass];      // chunk-sort tile (items per workgroup)
  uint32_t P[kNClass];      // merge tile
  uint32_t chunk[kNClass];  // odd-even chunk size
  uint32_t fan[kNClass];    // runs merged per HBM pass: 2 or 4
};

// A workgroup's work: from the device-side segment lists, or one segment given
// directly by the host (the per-bucket-launch form).  With chunks_only (direct
// work only) the chunk sort writes each chunk's sorted indices and stops: the
// slaves' step of section 4 without the master's merge.
struct TileWork {
  uint32_t direct;
  uint32_t base, n, m;
  uint32_t chunks_only;
};

// ---------------------------------------------------------------- wave tools
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes whose BITS-bit key equals this lane's (valid lanes only).  Per bit b,
// `mine` is all ones where the lane's bit is set and the ballot holds the
// lanes with it set, so (ballot ^ mine) are the lanes that differ from this
// one on bit b; v_bitop3 (0xF6: a | (b ^ c)) gathers them over the bits, two
// instructions a bit for the 64-lane mask.  The empty asm keeps `mine` the
// value the ballot compares, rather than a second shift of the key.
template <int BITS>
__device__ inline uint64_t match_mask(uint32_t key, bool valid) {
  uint32_t dlo = 0, dhi = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    uint32_t mine = (uint32_t)__builtin_amdgcn_sbfe((int)key, b, 1);
    asm volatile("" : "+v"(mine));
    const uint64_t bb = __ballot(mine != 0u);
    dlo = __builtin_amdgcn_bitop3_b32(dlo, (uint32_t)bb, mine, 0xF6);
    dhi = __builtin_amdgcn_bitop3_b32(dhi, (uint32_t)(bb >> 32), mine, 0xF6);
  }
  return __ballot(valid) & ~(((uint64_t)dhi << 32) | dlo);
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan over the workgroup; s_tmp holds NT/64 words.  Ends with a
// barrier, so s_tmp may be reused at once.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_tmp, uint32_t& total) {
  constexpr int NW = NT / 64;
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    uint32_t x = lane < NW ? s_tmp[lane] : 0u;
    x = wave_incl_scan(x);
    if (lane < NW) s_tmp[lane] = x;
  }
  __syncthreads();
  const uint32_t before = wave ? s_tmp[wave - 1] : 0u;
  total = s_tmp[NW - 1];
  __syncthreads();
  return before + incl - v;
}

// Largest k in [0, count) with prefix[k] <= t, for non-decreasing prefix with
// prefix[0] <= t.  One wave, 64 probes per round.
__device__ inline uint32_t wave_find(const uint32_t* prefix, uint32_t count, uint32_t t) {
  const uint32_t lane = __lane_id();
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) >> 6;
    const uint32_t pos = lo + lane * step;
    const bool p = pos < hi && prefix[pos] <= t;
    const uint32_t c = max((uint32_t)__popcll(__ballot(p)), 1u);   // prefix[lo] <= t holds
    lo = lo + (c - 1) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Streaming loads (nontemporal hint) for inputs read once.
template <int NL>
__device__ inline Key<NL> gload_nt(const KeyBuf& b, size_t p) {
  Key<NL> v;
#pragma unroll
  for (int q = 0; q < NL; ++q) v.k[q] = __builtin_nontemporal_load(b.k[q] + p);
  v.idx = __builtin_nontemporal_load(b.idx + p);
  return v;
}
template <>
__device__ inline Key<0> gload_nt<0>(const KeyBuf& b, size_t p) {
  Key<0> v;
  v.k = __builtin_nontemporal_load(b.k[0] + p);
  return v;
}

// Streaming stores (nontemporal hint) for outputs that the next kernel reads
// only after the whole level has been written.
template <int NL>
__device__ inline void gstore_nt(const KeyBuf& b, size_t p, const Key<NL>& v) {
#pragma unroll
  for (int q = 0; q < NL; ++q) __builtin_nontemporal_store(v.k[q], b.k[q] + p);
  __builtin_nontemporal_store(v.idx, b.idx + p);
}
template <>
__device__ inline void gstore_nt<0>(const KeyBuf& b, size_t p, const Key<0>& v) {
  __builtin_nontemporal_store(v.k, b.k[0] + p);
}

// Neighbour exchange across the whole wave with DPP wavefront shifts (GFX9
// data-parallel primitives, a VALU move, no LDS round trip): kDppNext gives
// lane i the value of lane i+1, kDppPrev that of lane i-1; the lane with no
// such neighbour (63, resp. 0) keeps its own value.
constexpr int kDppNext = 0x130;   // wavefront shift left by one lane
constexpr int kDppPrev = 0x138;   // wavefront shift right by one lane
// Quad permutes (controls below 0x100) write every lane, so they need no
// old value kept (no copy before the move).
template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t v) {
  if constexpr (CTRL < 0x100)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline uint64_t dpp64(uint64_t v) {
  return ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}
template <int CTRL, int NL>
__device__ inline Key<NL> key_dpp(const Key<NL>& v) {
  Key<NL> r;
#pragma unroll
  for (int q = 0; q < NL; ++q) r.k[q] = dpp64<CTRL>(v.k[q]);
  r.idx = dpp32<CTRL>(v.idx);
  return r;
}
template <int CTRL>
__device__ inline Key<0> key_dpp(const Key<0>& v) {
  Key<0> r;
  r.k = dpp64<CTRL>(v.k);
  return r;
}

// ---------------------------------------------------------------- LDS tile
// Structure-of-arrays tile of CAP keys.  One pad slot every 2^PADSH items
// keeps a thread's consecutive items (blocked layout) off its neighbours'
// banks.
template <int NL, int CAP, int PADSH = 4>
struct LdsTile {
  using value_type = Key<NL>;
  static constexpr int kPadded = CAP + (CAP >> PADSH);
  static constexpr int kLanes = NL ? NL : 1;
  uint64_t k[kLanes][kPadded];
  uint32_t idx[NL ? kPadded : 1];

  __device__ static int pos(int i) {
    const uint32_t u = (uint32_t)i;   // i >= 0: a logical shift
    return (int)(u + (u >> PADSH));
  }
  __device__ Key<NL> get(int i) const {
    const int p = pos(i);
    Key<NL> v;
#pragma unroll
    for (int q = 0; q < NL; ++q) v.k[q] = k[q][p];
    v.idx = idx[p];
    return v;
  }
  __device__ void put(int i, const Key<NL>& v) {
    const int p = pos(i);
#pragma unroll
    for (int q = 0; q < NL; ++q) k[q][p] = v.k[q];
    idx[p] = v.idx;
  }
};
template <int CAP, int PADSH>
struct LdsTile<0, CAP, PADSH> {
  using value_type = Key<0>;
  static constexpr int kPadded = CAP + (CAP >> PADSH);
  uint64_t k[kPadded];
  __device__ static int pos(int i) {
    const uint32_t u = (uint32_t)i;
    return (int)(u + (u >> PADSH));
  }
  // Byte offset of item i, (i + i/2^PADSH) * 8: one shift and one
  // add-and-scale (i >= 0).
  __device__ static uint32_t boff(int i) {
    const uint32_t u = (uint32_t)i;
    return (u + (u >> PADSH)) << 3;
  }
  __device__ Key<0> get(int i) const {
    Key<0> v;
    v.k = *(const uint64_t*)((const char*)k + boff(i));
    return v;
  }
  __device__ void put(int i, const Key<0>& v) { *(uint64_t*)((char*)k + boff(i)) = v.k; }
};

// ---------------------------------------------------------------- tagged keys
// A key with a small tag compared first.  Several short segments packed into
// one tile carry their ordinal in the tile as the tag, so sorting the tile by
// (tag, key) sorts every segment in place.
template <int NL>
struct TKey {
  Key<NL> k;
  uint32_t tag;
};

template <int NL, int CAP, int PADSH = 4>
struct TLdsTile {
  using value_type = TKey<NL>;
  LdsTile<NL, CAP, PADSH> t;
  uint32_t tag[LdsTile<NL, CAP, PADSH>::kPadded];
  __device__ TKey<NL> get(int i) const {
    TKey<NL> v;
    v.k = t.get(i);
    v.tag = tag[LdsTile<NL, CAP, PADSH>::pos(i)];
    return v;
  }
  __device__ void put(int i, const TKey<NL>& v) {
    t.put(i, v.k);
    tag[LdsTile<NL, CAP, PADSH>::pos(i)] = v.tag;
  }
};

// Element operations, overloaded for plain and tagged keys.
template <int NL>
__device__ inline bool e_less(const Key<NL>& a, const Key<NL>& b) { return key_less<NL>(a, b); }
template <int NL>
__device__ inline bool e_less(const TKey<NL>& a, const TKey<NL>& b) {
  return (a.tag < b.tag) | ((a.tag == b.tag) & key_less<NL>(a.k, b.k));
}
template <int NL>
__device__ inline Key<NL> e_select(bool c, const Key<NL>& x, const Key<NL>& y) { return key_select<NL>(c, x, y); }
template <int NL>
__device__ inline TKey<NL> e_select(bool c, const TKey<NL>& x, const TKey<NL>& y) {
  TKey<NL> r;
  r.k = key_select<NL>(c, x.k, y.k);
  r.tag = c ? x.tag : y.tag;
  return r;
}
template <int NL>
__device__ inline void e_set_sentinel(Key<NL>& v) { v = key_sentinel<NL>(); }
template <int NL>
__device__ inline void e_set_sentinel(TKey<NL>& v) {
  v.k = key_sentinel<NL>();
  v.tag = ~0u;
}
template <int NL>
__device__ inline void e_set_fill(Key<NL>& v) { v = key_fill<NL>(); }
template <int NL>
__device__ inline void e_set_fill(TKey<NL>& v) {
  v.k = key_fill<NL>();
  v.tag = ~0u;
}
template <class K>
__device__ inline K e_sentinel() {
  K v;
  e_set_sentinel(v);
  return v;
}
template <int CTRL, int NL>
__device__ inline Key<NL> e_dpp(const Key<NL>& v) { return key_dpp<CTRL>(v); }
template <int CTRL, int NL>
__device__ inline TKey<NL> e_dpp(const TKey<NL>& v) {
  TKey<NL> r;
  r.k = key_dpp<CTRL>(v.k);
  r.tag = dpp32<CTRL>(v.tag);
  return r;
}
// Compare-exchange: afterwards a <= b.  Returns whether they were exchanged.
template <class K>
__device__ inline bool e_cmp_xchg(K& a, K& b) {
  const bool sw = e_less(b, a);
  const K lo = e_select(sw, b, a);
  const K hi = e_select(sw, a, b);
  a = lo;
  b = hi;
  return sw;
}

}  // namespace sw
